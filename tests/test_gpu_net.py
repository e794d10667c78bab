"""GPU parity of the learned preconditioner (the parallel-transport network,
its loss and weight gradients, Adam training, training pairs and flexible
CG) against the network oracle, through the C ABI.

Tolerances: the network runs in FP32 with bfloat16 weights; the oracle uses
the same bfloat16-rounded weight values and the FP32-rounded inputs in FP64,
so the remaining difference is FP32 accumulation over 20 terms x at most 8
channels per layer through the 2 x 3 layers of B^dag B: each layer adds a
few 2^-24 relative errors of its largest terms, about 1e-6 after six layers,
so 1e-5 relative (max-norm) for outputs, 1e-4 for the loss and the weight
gradients (sums over all sites of FP32 products, and FP32 applications of
A = M^dag M in the residual loss).
Solves: FP64 true residual <= 1e-10, re-measured by the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import eo, nn
from oracle.dwf import Action, System, H_system
from oracle.lattice import restrict, norm2, dagger, shift
from paper_1706_05843_amd import eofa, synth

pytestmark = pytest.mark.gpu

M5, B5, C5 = 1.8, 1.5, 0.5
DIMS, LS = (4, 4, 4, 4), 4
BC = (1, 1, 1, -1)
CHANS = [1, 4, 4, 1]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def make(dims=DIMS, Ls=LS, eps=0.5, seed=11, U=None):
    act = Action(dims, Ls, M5, B5, C5, BC)
    if U is None:
        U = synth.gauge_field(dims, eps, seed)
    ctx = eofa.Context(eofa.make_action(dims, Ls, M5, B5, C5, BC), dev(U))
    return act, U, ctx


def f32(a):
    return a.astype(np.complex64).astype(np.complex128)


def to_packed(ctx, full_odd, n=1):
    """Canonical fields [n, Ls, T, Z, Y, X, 4, 3] -> n consecutive packed FP32 odd half-fields."""
    b = ctx.packed_bytes(eofa.FP32)
    out = torch.empty(n * b, dtype=torch.uint8, device="cuda")
    f = dev(full_odd)
    for k in range(n):
        ctx.eofa_pack(f[k:k + 1].contiguous(), out[k * b:(k + 1) * b], 1, eofa.FP32)
    return out


def from_packed(ctx, packed, n=1):
    b = ctx.packed_bytes(eofa.FP32)
    outs = []
    for k in range(n):
        full = torch.zeros(ctx.full_shape(1), dtype=torch.complex128, device="cuda")
        ctx.eofa_unpack(packed[k * b:(k + 1) * b], full, 1, eofa.FP32)
        outs.append(host(full)[0])
    return np.stack(outs)


def rand_weights(chans, seed, scale=0.4):
    rng = np.random.default_rng(seed)
    T = nn.NTERMS
    return [scale * (rng.standard_normal((T, co, ci)) + 1j * rng.standard_normal((T, co, ci)))
            for ci, co in zip(chans[:-1], chans[1:])]


def odd_field(dims, Ls, seed, n=1):
    return np.stack([restrict(synth.fermion(dims, Ls, seed + k), dims, 1) for k in range(n)])


def test_forward_matches_oracle():
    act, U, ctx = make()
    net = eofa.Net(ctx, CHANS, seed=1)
    W = rand_weights(CHANS, 2)
    net.set_weights(W)
    Wb = [nn.bf16_round(w.astype(np.complex64).astype(np.complex128)) for w in W]
    r = f32(odd_field(DIMS, LS, 30))
    pin = to_packed(ctx, r)
    pout = ctx.new_packed(eofa.FP32)
    net.apply(ctx, pin, pout)
    got = from_packed(ctx, pout)[0]
    ref = nn.forward(U, Wb, r[0], DIMS, BC)[0]
    assert rel(got, ref) < 1e-5
    # even sites of the output are not produced (odd half-field only)
    assert np.abs(restrict(got, DIMS, 0)).max() == 0.0


def test_weights_roundtrip_and_bf16_use():
    act, U, ctx = make()
    net = eofa.Net(ctx, [1, 3, 1], seed=4)
    W = rand_weights([1, 3, 1], 5)
    net.set_weights(W)
    back = net.get_weights()
    for a, b in zip(back, W):
        assert np.abs(a - b.astype(np.complex64)).max() == 0.0  # FP32 master copy


def test_loss_and_gradients_match_oracle():
    act, U, ctx = make(seed=12)
    net = eofa.Net(ctx, CHANS, seed=3)
    W = rand_weights(CHANS, 6)
    net.set_weights(W)
    Wb = [nn.bf16_round(w.astype(np.complex64).astype(np.complex128)) for w in W]
    npairs = 3
    r = f32(odd_field(DIMS, LS, 40, npairs))
    e = f32(odd_field(DIMS, LS, 50, npairs))
    loss, grads = net.loss_grad(ctx, to_packed(ctx, r, npairs), to_packed(ctx, e, npairs), npairs)
    Lref, gref = nn.loss_and_grads(U, Wb, [(r[k], e[k]) for k in range(npairs)], DIMS, BC)
    assert abs(loss - Lref) < 1e-5 * Lref
    for g, gr in zip(grads, gref):
        assert rel(g, gr) < 1e-4


def test_residual_loss_and_gradients_match_oracle():
    """1 - |<A N(r), r>|^2/(|A N(r)|^2 |r|^2) with A = M^dag M applied in FP32 on
    the GPU, FP64 in the oracle."""
    act, U, ctx = make(seed=19)
    sysm = System(0.2, 0.0, 0.0, 0.0, 1)
    net = eofa.Net(ctx, CHANS, seed=3)
    W = rand_weights(CHANS, 26, scale=0.2)
    net.set_weights(W)
    Wb = [nn.bf16_round(w.astype(np.complex64).astype(np.complex128)) for w in W]
    npairs = 2
    r = f32(odd_field(DIMS, LS, 140, npairs))
    loss, grads = net.loss_grad(ctx, to_packed(ctx, r, npairs), None, npairs, system=sysm)
    S = eo.SchurSystem(act, U, sysm)
    A = lambda x: S.mhat_adj(S.mhat(x))
    Lref, gref = nn.residual_loss_and_grads(U, Wb, [r[k] for k in range(npairs)], A, DIMS, BC)
    assert abs(loss - Lref) < 1e-4 * Lref
    for g, gr in zip(grads, gref):
        assert rel(g, gr) < 1e-4


def test_gauge_covariance_on_gpu():
    """N[U^g](g r) = g N[U](r), each side evaluated by the GPU network."""
    act, U, ctx = make(seed=13)
    g = synth.gauge_transform(DIMS, seed=14)
    Ug = np.stack([g @ U[mu] @ dagger(shift(g, mu, +1)) for mu in range(4)])
    _, _, ctxg = make(U=np.ascontiguousarray(Ug))
    net = eofa.Net(ctx, CHANS, seed=5)
    net.set_weights(rand_weights(CHANS, 7))
    r = odd_field(DIMS, LS, 60)
    rot = lambda f: np.einsum("...ab,...sb->...sa", g, f)
    pa, pb = ctx.new_packed(eofa.FP32), ctx.new_packed(eofa.FP32)
    net.apply(ctxg, to_packed(ctxg, rot(r[0])[None]), pa)
    net.apply(ctx, to_packed(ctx, r), pb)
    a = from_packed(ctxg, pa)[0]
    b = rot(from_packed(ctx, pb)[0])
    assert rel(a, b) < 1e-5


def _pairs(ctx, sysm, npairs, stride, seed, first=0):
    phi = synth.fermion(ctx.dims, ctx.Ls, seed, nrhs=1)
    b = ctx.packed_bytes(eofa.FP32)
    r = torch.empty(npairs * b, dtype=torch.uint8, device="cuda")
    e = torch.empty(npairs * b, dtype=torch.uint8, device="cuda")
    rc, rec, its = ctx.eofa_cg_pairs(sysm, dev(phi), npairs, first, stride, 1e-12, 20000, r, e)
    assert rc == eofa.EOFA_OK
    return r, e, rec, its


def test_pairs_satisfy_normal_equation():
    """A e_k = r_k with A = M^dag M of the odd Schur system (oracle operator)."""
    act, U, ctx = make(seed=15)
    sysm = System(0.1, 0.0, 0.0, 0.0, 1)
    r, e, rec, its = _pairs(ctx, sysm, 4, 5, 70)
    assert rec == 4 and its > 15
    S = eo.SchurSystem(act, U, sysm)
    R, E = from_packed(ctx, r, rec), from_packed(ctx, e, rec)
    for k in range(rec):
        AE = S.mhat_adj(S.mhat(E[k]))
        # FP32 storage of e_k (2^-24 relative) is amplified by up to the condition number of A
        assert np.sqrt(norm2(AE - R[k]) / norm2(R[k])) < 1e-3, k
    # the first pair is the initial residual r_0 = M^dag b~ (x_0 = 0, e_0 = x*)
    from oracle.dwf import g5R5
    phi = synth.fermion(act.dims, act.Ls, 70, nrhs=1)[0]
    r0 = S.mhat_adj(S.schur_source(g5R5(phi)))
    assert rel(R[0], r0) < 2e-6


def test_training_reduces_loss():
    act, U, ctx = make(seed=16)
    sysm = System(0.1, 0.0, 0.0, 0.0, 1)
    r, e, rec, _ = _pairs(ctx, sysm, 16, 2, 80)
    net = eofa.Net(ctx, CHANS, seed=8, init_scale=0.5)
    hist = net.train(ctx, r, e, rec, epochs=30, batch=4, lr=3e-3)
    assert all(np.isfinite(hist))
    assert hist[-1] < 0.8 * hist[0]
    loss, _ = net.loss_grad(ctx, r, e, rec)
    assert loss / rec < hist[0]


def test_training_residual_loss_reduces_loss():
    act, U, ctx = make(seed=16)
    sysm = System(0.1, 0.0, 0.0, 0.0, 1)
    r, _, rec, _ = _pairs(ctx, sysm, 16, 2, 81)
    net = eofa.Net(ctx, CHANS, seed=8, init_scale=0.3)
    loss0, _ = net.loss_grad(ctx, r, None, rec, system=sysm)
    hist = net.train(ctx, r, None, rec, epochs=30, batch=4, lr=3e-3, system=sysm)
    assert all(np.isfinite(hist))
    loss1, _ = net.loss_grad(ctx, r, None, rec, system=sysm)
    print("residual loss per pair: untrained", loss0 / rec, "epochs", hist[0], hist[-1], "trained", loss1 / rec)
    assert loss1 < 0.9 * loss0 and loss1 / rec < 1.0


@pytest.mark.parametrize("which", ["identity", "trained", "zero"])
def test_fgcg_reaches_fp64_residual(which):
    act, U, ctx = make(seed=17)
    sysm = System(1.0, 0.04, 1.0, -1.0, +1)
    phi = synth.fermion(DIMS, LS, 90, nrhs=1)
    net = None
    if which != "identity":
        net = eofa.Net(ctx, CHANS, seed=9, init_scale=0.5)
        if which == "zero":
            net.set_weights([np.zeros((nn.NTERMS, co, ci)) for ci, co in zip(CHANS[:-1], CHANS[1:])])
        else:
            r, _, rec, _ = _pairs(ctx, sysm, 16, 2, 91)
            net.train(ctx, r, None, rec, epochs=20, batch=4, lr=3e-3, system=sysm)
    psi = torch.zeros_like(dev(phi))
    prm = eofa.make_params(tol=1e-10, precond=1, net=net)
    rc, st = ctx.eofa_cg_solve([sysm], dev(phi), psi, prm)
    assert rc == eofa.EOFA_OK and st[0]["converged"] == 1 and st[0]["true_resid"] <= 1e-10
    # a zero network cannot precondition: the solve must have fallen back to CGNR
    if which == "zero":
        assert st[0]["fell_back"] == 1
    elif which == "identity":
        assert st[0]["fell_back"] == 0
    sol = host(psi)[0]
    res = H_system(act, U, sysm, sol) - phi[0]
    assert np.sqrt(norm2(res) / norm2(phi[0])) < 1.05e-10
    print(which, "FGCG iterations", st[0]["iters"], "fell back", st[0]["fell_back"])


def test_fgcg_identity_iterations_match_cgnr():
    """Flexible CG with the identity is CG on the normal equations: same
    iteration count as the CGNR path within the polling granularity."""
    act, U, ctx = make(seed=18)
    sysm = System(0.1, 0.0, 0.0, 0.0, 1)
    phi = dev(synth.fermion(DIMS, LS, 95, nrhs=1))
    psi = torch.zeros_like(phi)
    rc, st_f = ctx.eofa_cg_solve([sysm], phi, psi, eofa.make_params(tol=1e-10, precond=1, check_every=1))
    assert rc == eofa.EOFA_OK
    rc, st_c = ctx.eofa_cg_solve([sysm], phi, torch.zeros_like(phi), eofa.make_params(tol=1e-10, check_every=1))
    assert rc == eofa.EOFA_OK
    assert abs(st_f[0]["iters"] - st_c[0]["iters"]) <= max(3, 0.1 * st_c[0]["iters"])


def test_network_is_hermitian_positive_on_gpu():
    """<a, N b> = <N a, b> and <a, N a> > 0 for the GPU network (N = B^dag B)."""
    act, U, ctx = make(seed=20)
    net = eofa.Net(ctx, CHANS, seed=5)
    net.set_weights(rand_weights(CHANS, 21, scale=0.3))
    a, b = odd_field(DIMS, LS, 150), odd_field(DIMS, LS, 151)
    pa, pb = ctx.new_packed(eofa.FP32), ctx.new_packed(eofa.FP32)
    net.apply(ctx, to_packed(ctx, a), pa)
    net.apply(ctx, to_packed(ctx, b), pb)
    Na, Nb = from_packed(ctx, pa)[0], from_packed(ctx, pb)[0]
    lhs, rhs = np.vdot(f32(a[0]), Nb), np.vdot(Na, f32(b[0]))
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)
    q = np.vdot(f32(a[0]), Na)
    assert q.real > 0 and abs(q.imag) < 1e-5 * q.real


def test_trained_network_beats_identity_on_held_out_field():
    """The purpose of the learned preconditioner: trained (residual loss) on
    CG residuals of one gauge field, flexible CG with N needs fewer
    iterations than flexible CG with the identity (plain CGNR) on a held-out
    source of that field and on a held-out field of the same ensemble
    (4^4 x Ls = 8, links exp(i 0.5 H), m1 = 0.04, m2 = 1.0)."""
    dims, Ls = (4, 4, 4, 4), 8
    sysm = System(1.0, 0.04, 1.0, -1.0, +1)
    act, U, ctx = make(dims, Ls, eps=0.5, seed=3000)
    b = ctx.packed_bytes(eofa.FP32)
    parts, n = [], 0
    for k in range(4):
        r, _, rec, _ = _pairs(ctx, sysm, 64, 3, 3100 + k)
        parts.append(r[:rec * b])
        n += rec
    R = torch.cat(parts)
    net = eofa.Net(ctx, [1, 4, 1], seed=1, init_scale=0.25)
    loss0, _ = net.loss_grad(ctx, R, None, n, system=sysm)
    hist = net.train(ctx, R, None, n, epochs=6, batch=16, lr=1e-2, system=sysm)
    assert all(np.isfinite(hist))

    def iters(c, seed, use_net):
        phi = dev(synth.fermion(dims, Ls, seed, nrhs=1))
        prm = eofa.make_params(tol=1e-10, precond=1, net=net if use_net else None, check_every=1)
        rc, st = c.eofa_cg_solve([sysm], phi, torch.zeros_like(phi), prm)
        assert rc == eofa.EOFA_OK and st[0]["converged"] == 1 and st[0]["true_resid"] <= 1e-10
        assert st[0]["fell_back"] == 0
        return st[0]["iters"]

    _, _, ctx1 = make(dims, Ls, eps=0.5, seed=4000)
    res = {"source": (iters(ctx, 3104, False), iters(ctx, 3104, True)),
           "field": (iters(ctx1, 4100, False), iters(ctx1, 4100, True))}
    print("residual loss per pair", loss0 / n, "->", hist[-1], "; FGCG iterations (identity, trained):", res)
    for ident, trained in res.values():
        assert trained <= 0.85 * ident


@pytest.mark.parametrize("window", [1, 8, 12])
def test_fgcg_windows_converge(window):
    """Flexible CG with the identity for several orthogonalisation windows
    (12 exercises two passes of the fused multi-direction kernels, at most 8
    directions each): each reaches the FP64 true residual, re-measured by the
    oracle, in about the iterations of CGNR (the identity makes every
    window's directions conjugate in exact arithmetic)."""
    act, U, ctx = make(seed=22)
    sysm = System(0.1, 0.0, 0.0, 0.0, 1)
    phi = synth.fermion(DIMS, LS, 96, nrhs=1)
    psi = torch.zeros_like(dev(phi))
    prm = eofa.make_params(tol=1e-10, precond=1, fcg_window=window, check_every=1)
    rc, st = ctx.eofa_cg_solve([sysm], dev(phi), psi, prm)
    assert rc == eofa.EOFA_OK and st[0]["converged"] == 1 and st[0]["fell_back"] == 0
    rc, st_c = ctx.eofa_cg_solve([sysm], dev(phi), torch.zeros_like(psi), eofa.make_params(tol=1e-10, check_every=1))
    assert abs(st[0]["iters"] - st_c[0]["iters"]) <= max(3, 0.1 * st_c[0]["iters"])
    sol = host(psi)[0]
    res = H_system(act, U, sysm, sol) - phi[0]
    assert np.sqrt(norm2(res) / norm2(phi[0])) < 1.05e-10
