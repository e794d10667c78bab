"""Pins of the network oracle: finite-difference gradients, the adjoint
identity, the layer's terms against the Wilson hop and explicit shifts,
N = B^dag B Hermitian positive semi-definite, gauge covariance, and flexible
CG with an exact preconditioner."""
import numpy as np

from oracle import nn, eo
from oracle.dwf import Action, System, g5R5
from oracle.lattice import restrict, vdot, norm2, dagger, shift, hop, P_PLUS, P_MINUS
from paper_1706_05843_amd import synth

DIMS, LS = (2, 2, 4, 2), 2
BC = (1.0, 1.0, 1.0, -1.0)


def _weights(chans, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    T = nn.NTERMS
    return [scale * (rng.standard_normal((T, co, ci)) + 1j * rng.standard_normal((T, co, ci)))
            for ci, co in zip(chans[:-1], chans[1:])]


def _field(seed, C=None):
    f = synth.fermion(DIMS, LS, seed)
    return f if C is None else np.stack([synth.fermion(DIMS, LS, seed + k) for k in range(C)])


def test_layer_adjoint_identity():
    U = synth.gauge_field(DIMS, 0.8, seed=1)
    W = _weights([3, 2], 2)[0]
    X, G = _field(10, 3), _field(20, 2)
    lhs = vdot(G, nn.layer(U, W, X, BC))
    rhs = vdot(nn.layer_adjoint(U, W, G, BC), X)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gradients_match_finite_differences():
    U = synth.gauge_field(DIMS, 0.8, seed=3)
    Ws = _weights([1, 2, 2, 1], 4)
    pairs = [(restrict(_field(30 + k), DIMS, 1), restrict(_field(40 + k), DIMS, 1)) for k in range(2)]
    L, grads = nn.loss_and_grads(U, Ws, pairs, DIMS, BC)
    rng = np.random.default_rng(5)
    h = 1e-6
    for layer_k in range(3):
        for _ in range(3):
            idx = tuple(int(rng.integers(0, n)) for n in Ws[layer_k].shape)
            for comp, unit in (("re", 1.0), ("im", 1j)):
                Wp = [w.copy() for w in Ws]
                Wm = [w.copy() for w in Ws]
                Wp[layer_k][idx] += unit * h
                Wm[layer_k][idx] -= unit * h
                fd = (nn.loss_and_grads(U, Wp, pairs, DIMS, BC)[0] - nn.loss_and_grads(U, Wm, pairs, DIMS, BC)[0]) / (2 * h)
                g = grads[layer_k][idx]
                an = 2 * (g.real if comp == "re" else g.imag)
                assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (layer_k, idx, comp, fd, an)


def test_residual_loss_gradients_match_finite_differences():
    """Residual loss sum_p min_c |c A N(r_p) - r_p|^2/|r_p|^2 with A = M^dag M of a Schur system."""
    act = Action(DIMS, LS, 1.8, 1.5, 0.5, BC)
    U = synth.gauge_field(DIMS, 0.8, seed=21)
    S = eo.SchurSystem(act, U, System(0.2))
    A = lambda x: S.mhat_adj(S.mhat(x))
    Ws = _weights([1, 2, 1], 22, scale=0.2)
    rs = [restrict(_field(130 + k), DIMS, 1) for k in range(2)]
    L, grads = nn.residual_loss_and_grads(U, Ws, rs, A, DIMS, BC)
    # the loss is the least-squares misfit min_c |c A N r - r|^2 / |r|^2, the
    # best scale taken by a library least-squares solve
    Lref = 0.0
    for r in rs:
        a = A(nn.forward(U, Ws, r, DIMS, BC)[0]).ravel()
        c = np.linalg.lstsq(a[:, None], r.ravel(), rcond=None)[0][0]
        Lref += norm2(c * a - r.ravel()) / norm2(r)
    assert abs(L - Lref) < 1e-10 * max(Lref, 1e-3)
    rng = np.random.default_rng(23)
    h = 1e-6
    for layer_k in range(2):
        for _ in range(3):
            idx = tuple(int(rng.integers(0, n)) for n in Ws[layer_k].shape)
            for comp, unit in (("re", 1.0), ("im", 1j)):
                Wp = [w.copy() for w in Ws]
                Wm = [w.copy() for w in Ws]
                Wp[layer_k][idx] += unit * h
                Wm[layer_k][idx] -= unit * h
                fd = (nn.residual_loss_and_grads(U, Wp, rs, A, DIMS, BC)[0]
                      - nn.residual_loss_and_grads(U, Wm, rs, A, DIMS, BC)[0]) / (2 * h)
                g = grads[layer_k][idx]
                an = 2 * (g.real if comp == "re" else g.imag)
                assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (layer_k, idx, comp, fd, an)


def test_gauge_covariance():
    """N[U^g](g r) = g N[U](r)."""
    U = synth.gauge_field(DIMS, 0.8, seed=6)
    g = synth.gauge_transform(DIMS, seed=7)
    Ug = np.stack([g @ U[mu] @ dagger(shift(g, mu, +1)) for mu in range(4)])
    Ws = _weights([1, 2, 1], 8)
    r = restrict(_field(50), DIMS, 1)
    rot = lambda f: np.einsum("...ab,...sb->...sa", g, f)
    a = nn.forward(Ug, Ws, rot(r), DIMS, BC)[0]
    b = rot(nn.forward(U, Ws, r, DIMS, BC)[0])
    assert np.abs(a - b).max() < 1e-14 * np.abs(b).max()


def test_fcg_with_exact_preconditioner_and_identity():
    """FCG with N = A^-1 converges in one step; with N = 1 it is CG."""
    act = Action((2, 2, 2, 2), 4, 1.8, 1.5, 0.5, BC)
    U = synth.gauge_field(act.dims, 0.3, seed=9)
    S = eo.SchurSystem(act, U, System(0.04))
    bt = S.schur_source(g5R5(synth.fermion(act.dims, act.Ls, seed=60)))
    A = lambda x: S.mhat_adj(S.mhat(x))
    rhs = S.mhat_adj(bt)
    x_cg, n_cg, _ = eo.cgnr(S.mhat, S.mhat_adj, bt, tol=1e-11)
    x_f, n_f = nn.fcg(A, lambda r: r, rhs, tol=1e-11)
    assert np.sqrt(norm2(x_f - x_cg) / norm2(x_cg)) < 1e-8
    assert abs(n_f - n_cg) <= 2
    x_e, n_e = nn.fcg(A, lambda r: _solve_normal(S, r), rhs, tol=1e-10)
    assert n_e <= 2


def _solve_normal(S, r):
    """A^-1 r for A = M^dag M by CG on A (r is a normal-equation residual)."""
    x = np.zeros_like(r)
    rr = r.copy()
    p = rr.copy()
    rs = norm2(rr)
    for _ in range(2000):
        q = S.mhat_adj(S.mhat(p))
        a = rs / vdot(p, q).real
        x += a * p
        rr -= a * q
        rn = norm2(rr)
        if rn < 1e-28 * norm2(r):
            break
        p = rr + (rn / rs) * p
        rs = rn
    return x


def test_bf16_rounding():
    x = np.array([1.0 + 2.0 ** -9, 1.0 + 3 * 2.0 ** -9, -3.14159265, 1e-3])
    r = nn.bf16_round(x + 0j).real
    assert r[0] == 1.0 and r[1] == 1.0 + 2.0 ** -7 and abs(r[2] + 3.140625) < 1e-12
    assert abs(r[3] - 1e-3) < 1e-3 * 2 ** -8


def test_hop_terms_make_the_wilson_hop():
    """With weights -1/2 (1) and +1/2 (gamma_mu) on the forward transports and
    -1/2, -1/2 on the backward ones the layer is the Wilson hop
    -1/2 sum_mu [(1 - g_mu) T_{+mu} + (1 + g_mu) T_{-mu}] (lattice.hop, pinned
    by brute force); the site-local and s terms are explicit projections and
    cyclic shifts."""
    U = synth.gauge_field(DIMS, 0.8, seed=11)
    X = _field(70, 1)
    W = np.zeros((nn.NTERMS, 1, 1), dtype=np.complex128)
    for mu in range(4):
        W[2 + mu], W[10 + mu] = -0.5, 0.5
        W[6 + mu], W[14 + mu] = -0.5, -0.5
    y = nn.layer(U, W, X, BC)[0]
    ref = hop(U, X[0], BC)
    assert np.abs(y - ref).max() < 1e-14 * np.abs(ref).max()
    W = np.zeros((nn.NTERMS, 1, 1), dtype=np.complex128)
    W[0], W[1], W[18], W[19] = 2.0, -1.0, 0.5j, 3.0
    y = nn.layer(U, W, X, BC)[0]
    f = X[0]
    sp = lambda m, g: np.einsum("st,...tc->...sc", m, g)
    ref = (2.0 * sp(P_PLUS, f) - sp(P_MINUS, f) + 0.5j * sp(P_PLUS, np.roll(f, 1, axis=0))
           + 3.0 * sp(P_MINUS, np.roll(f, -1, axis=0)))
    assert np.abs(y - ref).max() < 1e-14


def test_network_hermitian_positive():
    """<a, N b> = <N a, b> and <a, N a> = |B a|^2 >= 0 for N = B^dag B."""
    U = synth.gauge_field(DIMS, 0.8, seed=12)
    Ws = _weights([1, 3, 2, 1], 13)
    a, b = restrict(_field(80), DIMS, 1), restrict(_field(81), DIMS, 1)
    Na, Nb = nn.forward(U, Ws, a, DIMS, BC)[0], nn.forward(U, Ws, b, DIMS, BC)[0]
    lhs, rhs = vdot(a, Nb), vdot(Na, b)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    Ba = a[None]
    for W in Ws:
        Ba = nn.layer(U, W, Ba, BC)
    q = vdot(a, Na)
    assert abs(q.imag) < 1e-12 * abs(q) and abs(q.real - norm2(Ba)) < 1e-12 * norm2(Ba)
