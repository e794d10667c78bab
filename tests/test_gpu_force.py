"""GPU parity of the link derivative of Dhop and the EOFA pseudofermion force
(Sec. IV C, eqn eofa_force) against the force oracle, through the C ABI.

* eofa_dhop_derivative: Tr(T^a y_mu(x)) equals the oracle's derivative of
  a^dag Dhop b along e^{s T^a} U_mu(x), all 8 generators, sampled links
  including the lattice corners (boundary phases), FP64: 1e-13 relative.
* eofa_force on 2^4 x Ls=4 against the oracle's eqn eofa_force with dense-LU
  solves at every link (the oracle's formula is itself pinned to central
  differences of the action in the CPU suite): the GPU solves to a 1e-12 true
  residual, so the force agrees to 1e-9 relative (condition number x tol).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import force, reference, eo
from oracle.dwf import Action
from paper_1706_05843_amd import eofa, synth

pytestmark = pytest.mark.gpu

M5, B5, C5 = 1.8, 1.5, 0.5
BC = (1, 1, 1, -1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def make(dims, Ls, eps, seed):
    act = Action(dims, Ls, M5, B5, C5, BC)
    U = synth.gauge_field(dims, eps, seed)
    ctx = eofa.Context(eofa.make_action(dims, Ls, M5, B5, C5, BC), dev(U))
    return act, U, ctx


def links_sample(dims, n, seed):
    rng = np.random.default_rng(seed)
    out = [((dims[0] - 1, dims[1] - 1, dims[2] - 1, dims[3] - 1), mu) for mu in range(4)]
    out += [((0, 0, 0, 0), mu) for mu in range(4)]
    while len(out) < n:
        out.append((tuple(int(rng.integers(0, L)) for L in dims), int(rng.integers(0, 4))))
    return out


@pytest.mark.parametrize("dims,Ls", [((4, 4, 4, 4), 4), ((2, 4, 2, 6), 2)])
def test_dhop_derivative_matches_oracle(dims, Ls):
    act, U, ctx = make(dims, Ls, 0.6, 31)
    a = synth.fermion(dims, Ls, 32)
    b = synth.fermion(dims, Ls, 33)
    y = torch.zeros(ctx.gauge_shape(), dtype=torch.complex128, device="cuda")
    ctx.eofa_dhop_derivative(dev(a), dev(b), y)
    Y = host(y)
    T = force.generators()
    got, ref = [], []
    for x, mu in links_sample(dims, 20, 34):
        Ym = Y[mu, x[3], x[2], x[1], x[0]]
        for k in range(8):
            got.append(np.trace(T[k] @ Ym))
            ref.append(force.dhop_derivative(U, a, b, BC, x, mu, T[k]))
    got, ref = np.array(got), np.array(ref)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


def test_force_matches_oracle_every_link():
    dims, Ls = (2, 2, 2, 2), 4
    act, U, ctx = make(dims, Ls, 0.5, 41)
    m1, m2 = 0.1, 0.6
    phi = synth.fermion(dims, Ls, 42)
    F = torch.zeros(ctx.gauge_shape(), dtype=torch.complex128, device="cuda")
    rc, st = ctx.eofa_force(m1, m2, dev(phi), F, eofa.make_params(tol=1e-12))
    assert rc == eofa.EOFA_OK and all(s["true_resid"] <= 1e-12 for s in st)
    Fg = host(F)
    solve = lambda sys, rhs: reference.solve_dense(act, U, sys, rhs)
    links = [((x, y, z, t), mu) for t in range(2) for z in range(2) for y in range(2) for x in range(2)
             for mu in range(4)]
    Fa = force.force_formula(act, U, m1, m2, phi, solve, links)
    ref = force.force_matrix(Fa)
    got = np.stack([Fg[mu, x[3], x[2], x[1], x[0]] for x, mu in links])
    assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max()
    # traceless anti-Hermitian
    assert np.abs(got + np.conj(np.transpose(got, (0, 2, 1)))).max() < 1e-14 * np.abs(got).max()
    assert np.abs(np.einsum("nii->n", got)).max() < 1e-14 * np.abs(got).max()


def test_force_sampled_on_4x4x4x8():
    dims, Ls = (4, 4, 4, 8), 8
    act, U, ctx = make(dims, Ls, 0.3, 51)
    m1, m2 = 0.04, 1.0
    phi = synth.fermion(dims, Ls, 52)
    F = torch.zeros(ctx.gauge_shape(), dtype=torch.complex128, device="cuda")
    rc, st = ctx.eofa_force(m1, m2, dev(phi), F, eofa.make_params(tol=1e-12, inner_prec=eofa.FP32))
    assert rc == eofa.EOFA_OK
    Fg = host(F)

    def solve(sys, rhs):
        return eo.solve_mirror(act, U, sys, rhs, tol=1e-13)["psi"]

    links = links_sample(dims, 12, 53)
    Fa = force.force_formula(act, U, m1, m2, phi, solve, links)
    ref = force.force_matrix(Fa)
    got = np.stack([Fg[mu, x[3], x[2], x[1], x[0]] for x, mu in links])
    assert np.abs(got - ref).max() < 1e-8 * np.abs(ref).max()
