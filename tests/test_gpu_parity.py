"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Tolerances: FP64 kernels 1e-13 relative (max-norm against the oracle's max);
FP32 storage 2e-6; FP16 storage with per-site scale 4e-3 (half precision has
a 2^-11 relative spacing and a hop sums 8 neighbours). Solves: mirror mode
(fixed iteration count equal to the oracle's) agrees to 1e-12 relative in the
2-norm; converged solves reach an FP64 true residual <= 1e-10, which the
oracle re-measures independently on the H form of the system.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import action as oaction, eo, site
from oracle.dwf import Action, System, Dtilde_op, H_system, apply_s, g5R5
from oracle import fifth
from oracle.lattice import hop, restrict, norm2
from paper_1706_05843_amd import eofa, synth

pytestmark = pytest.mark.gpu

M5, B5, C5 = 1.8, 1.5, 0.5
M1, M2 = 0.04, 1.0
TOL = {eofa.FP64: 1e-13, eofa.FP32: 2e-6, eofa.FP16S: 4e-3}
SYSTEMS = {
    "chi1": System(M1, M1, M2, 0.0, -1),
    "chi2": System(M2, M1, M2, -1.0, +1),
    "lh": System(M1, M1, M2, -0.5, -1),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def make(dims, Ls, eps, seed, bc=(1, 1, 1, -1)):
    act = Action(dims, Ls, M5, B5, C5, bc)
    U = synth.unit_gauge(dims) if eps == 0 else synth.gauge_field(dims, eps, seed)
    ctx = eofa.Context(eofa.make_action(dims, Ls, M5, B5, C5, bc), dev(U))
    return act, U, ctx


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def rel2(a, b):
    return np.sqrt(norm2(a - b) / norm2(b))


def gpu_dslash(ctx, systems, psi, out_parity, dagger, prec):
    n = psi.shape[0]
    f = dev(psi)
    pin, pout = ctx.new_packed(prec, n), ctx.new_packed(prec, n)
    ctx.eofa_pack(f, pin, 1 - out_parity, prec, n)
    ctx.eofa_dslash(systems, pin, pout, out_parity, dagger, prec, n)
    out = torch.zeros_like(f)
    ctx.eofa_unpack(pout, out, out_parity, prec, n)
    return host(out)


def oracle_dslash(act, U, m, psi, out_parity, dagger):
    x = restrict(psi, act.dims, 1 - out_parity)
    if dagger:
        y = Dtilde_op(act, m, hop(U, x, act.bc, adjoint=True), transpose=True)
    else:
        y = hop(U, Dtilde_op(act, m, x), act.bc)
    return restrict(y, act.dims, out_parity)


# --- pack / unpack -----------------------------------------------------------

@pytest.mark.parametrize("prec", [eofa.FP64, eofa.FP32, eofa.FP16S])
def test_pack_roundtrip(prec):
    act, U, ctx = make((4, 2, 2, 6), 6, 0.5, 1)
    psi = synth.fermion(act.dims, act.Ls, seed=2, nrhs=2)
    f = dev(psi)
    out = torch.zeros_like(f)
    for parity in (0, 1):
        p = ctx.new_packed(prec, 2)
        ctx.eofa_pack(f, p, parity, prec, 2)
        ctx.eofa_unpack(p, out, parity, prec, 2)
    got = host(out)
    if prec == eofa.FP64:
        assert np.array_equal(got, psi)
    else:
        assert rel(got, psi) < TOL[prec]
    # gamma_5 R5 on the way in (App. B: b = g5 R5 phi)
    p = ctx.new_packed(eofa.FP64, 2)
    out.zero_()
    for parity in (0, 1):
        ctx.eofa_pack(f, p, parity, eofa.FP64, 2, g5r5=1)
        ctx.eofa_unpack(p, out, parity, eofa.FP64, 2)
    ref = psi[:, ::-1].copy()
    ref[..., 2:, :] *= -1
    assert np.array_equal(host(out), ref)


# --- Dslash -----------------------------------------------------------------

# Ls = 16: the row form; other Ls a multiple of 4 (4, 8, 12, 20, 24, 28, 32):
# the generic form whose FP16S products run on the matrix cores, with 0, 4,
# 16 and 8 idle lanes per wave at Ls = 32, 20, 24, 28; Ls = 2, 6: the generic
# form with v_dot2 products. The larger lattices give several work-groups
# and a ragged last one.
LATTICES = [((2, 2, 2, 2), 4), ((4, 4, 4, 4), 8), ((4, 2, 6, 4), 6), ((6, 4, 2, 2), 12), ((2, 2, 2, 4), 16),
            ((2, 2, 2, 2), 2), ((2, 2, 2, 4), 20), ((4, 2, 2, 4), 24), ((2, 2, 2, 2), 28), ((2, 2, 4, 2), 32)]


@pytest.mark.parametrize("dims,Ls", LATTICES)
@pytest.mark.parametrize("prec", [eofa.FP64, eofa.FP32, eofa.FP16S])
def test_dslash_matches_oracle(dims, Ls, prec):
    act, U, ctx = make(dims, Ls, 0.5, 11)
    psi = synth.fermion(dims, Ls, seed=12, nrhs=1)
    for m in (0.04, 1.0):
        for par in (0, 1):
            for dag in (0, 1):
                got = gpu_dslash(ctx, [(m, 0.0, 0.0, 0.0, 1)], psi, par, dag, prec)[0]
                ref = oracle_dslash(act, U, m, psi[0], par, dag)
                assert rel(got, ref) < TOL[prec], (m, par, dag, rel(got, ref))


def test_dslash_free_field_and_adjoint():
    """U = 1 and the adjointness <a, D b> = <D^dag a, b> through the library."""
    act, U, ctx = make((4, 4, 4, 4), 8, 0.0, 0)
    a = synth.fermion(act.dims, act.Ls, seed=20, nrhs=1)
    b = synth.fermion(act.dims, act.Ls, seed=21, nrhs=1)
    sysl = [(0.04, 0.0, 0.0, 0.0, 1)]
    Db = gpu_dslash(ctx, sysl, b, 0, 0, eofa.FP64)[0]          # even <- odd
    Dda = gpu_dslash(ctx, sysl, a, 1, 1, eofa.FP64)[0]         # odd <- even (adjoint)
    lhs = np.vdot(restrict(a[0], act.dims, 0).ravel(), Db.ravel())
    rhs = np.vdot(Dda.ravel(), restrict(b[0], act.dims, 1).ravel())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    assert rel(Db, oracle_dslash(act, U, 0.04, b[0], 0, 0)) < 1e-13


def test_dslash_multi_rhs():
    """One launch, three right-hand sides with their own operator masses."""
    act, U, ctx = make((4, 4, 2, 4), 8, 0.5, 30)
    psi = synth.fermion(act.dims, act.Ls, seed=31, nrhs=3)
    ms = [0.04, 1.0, 0.3]
    for prec in (eofa.FP64, eofa.FP32):
        got = gpu_dslash(ctx, [(m, 0.0, 0.0, 0.0, 1) for m in ms], psi, 1, 0, prec)
        for r, m in enumerate(ms):
            assert rel(got[r], oracle_dslash(act, U, m, psi[r], 1, 0)) < TOL[prec]


# --- same-parity block ---------------------------------------------------------

@pytest.mark.parametrize("name", list(SYSTEMS))
@pytest.mark.parametrize("prec", [eofa.FP64, eofa.FP32])
def test_mooee_and_inverse(name, prec):
    act, U, ctx = make((4, 2, 2, 4), 8, 0.5, 40)
    sys = SYSTEMS[name]
    Ap, Am = fifth.mee_blocks(act.Ls, M5, act.c, act.d, sys.m_op, sys.beta, sys.chi, sys.m_a, sys.m_b)
    psi = synth.fermion(act.dims, act.Ls, seed=41, nrhs=1)
    f = dev(psi)
    pin, pout = ctx.new_packed(prec), ctx.new_packed(prec)
    sl = [sys]
    for dag in (0, 1):
        for inv in (0, 1):
            out = torch.zeros_like(f)
            for par in (0, 1):
                ctx.eofa_pack(f, pin, par, prec)
                (ctx.eofa_mooee_inv if inv else ctx.eofa_mooee)(sl, pin, pout, dag, prec)
                ctx.eofa_unpack(pout, out, par, prec)
            P, M = (np.linalg.inv(Ap), np.linalg.inv(Am)) if inv else (Ap, Am)
            if dag:
                P, M = P.T, M.T
            assert rel(host(out)[0], apply_s(P, M, psi[0])) < 10 * TOL[prec]


# --- solves --------------------------------------------------------------------

_ORACLE = {}


def oracle_c1(name):
    """Oracle mirror-mode solve at the small workload (4^4, Ls = 8, eps = 0.3)."""
    if name not in _ORACLE:
        act = Action((4, 4, 4, 4), 8, M5, B5, C5, (1, 1, 1, -1))
        U = synth.gauge_field(act.dims, 0.3, seed=1000)
        phi = synth.fermion(act.dims, act.Ls, seed=2000)
        out = eo.solve_mirror(act, U, SYSTEMS[name], phi, tol=1e-10)
        _ORACLE[name] = (act, U, phi, out)
    return _ORACLE[name]


@pytest.fixture(scope="module")
def c1ctx():
    act, U, phi, _ = oracle_c1("chi1")
    return eofa.Context(eofa.make_action(act.dims, act.Ls, M5, B5, C5, act.bc), dev(U))


_FLOOR = {}


def noise_floor(name, iters, draws=2):
    """How far the oracle's own mirror-mode solve moves after ``iters`` CGNR
    steps when every Schur-operator application is perturbed by half an ulp
    of relative noise (2^-53, independent per entry): the reproducibility
    limit of the FP64 recurrence itself. Largest over ``draws`` seeds of the
    solution difference and of the residual-space difference
    |(H + beta Delta P)(psi_noisy - psi)| / |phi|."""
    key = (name, iters)
    if key not in _FLOOR:
        act, U, phi, out = oracle_c1(name)
        sys_ = SYSTEMS[name]
        S = eo.SchurSystem(act, U, sys_)
        b = g5R5(phi)
        bt = S.schur_source(b)
        ref = eo.solve_mirror(act, U, sys_, phi, iters=iters)["psi"]
        worst_d, worst_r = 0.0, 0.0
        for seed in range(draws):
            rng = np.random.default_rng(7 + seed)

            def noisy(f):
                def g(x):
                    y = f(x)
                    return y * (1.0 + 2.0 ** -53 * rng.standard_normal(y.shape))
                return g
            xo, _, _ = eo.cgnr(noisy(S.mhat), noisy(S.mhat_adj), bt, iters=iters)
            psi = Dtilde_op(act, sys_.m_op, S.reconstruct(xo, b))
            worst_d = max(worst_d, rel2(psi, ref))
            worst_r = max(worst_r, np.sqrt(norm2(H_system(act, U, sys_, psi - ref)) / norm2(phi)))
        _FLOOR[key] = (worst_d, worst_r)
    return _FLOOR[key]


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_cg_mirror_mode_fp64(c1ctx, name):
    """Fixed iteration count: the same recurrences as the oracle.

    40 iterations: solution and residual-space differences <= 1e-12 for
    every system. The oracle's converged count: 1e-12 for the unshifted and
    heatbath systems; for the shifted system (H(m2) - Delta_+ P_+) the late
    CGNR steps amplify rounding by ~1e4-1e5, so there both differences are
    bounded by 3x the oracle's own spread under half-ulp noise per operator
    application (noise_floor; measured 5e-12 .. 1.4e-11), at least 1e-12."""
    act, U, phi, out = oracle_c1(name)
    for iters in (40, out["iters"]):
        ref = out["psi"] if iters == out["iters"] else eo.solve_mirror(act, U, SYSTEMS[name], phi, iters=iters)["psi"]
        psi = torch.zeros(c1ctx.full_shape(1), dtype=torch.complex128, device="cuda")
        rc, st = c1ctx.eofa_cg_solve([SYSTEMS[name]], dev(phi[None]), psi, eofa.make_params(fixed_iters=iters))
        assert st[0]["iters"] == iters
        got = host(psi)[0]
        d = rel2(got, ref)
        rdiff = np.sqrt(norm2(H_system(act, U, SYSTEMS[name], got - ref)) / norm2(phi))
        bd, br = 1e-12, 1e-12
        if iters == out["iters"] and name == "chi2":
            fd, fr = noise_floor(name, iters)
            bd, br = max(1e-12, 3.0 * fd), max(1e-12, 3.0 * fr)
            print(f"chi2 at {iters} iterations: gpu {d:.3e} / {rdiff:.3e}, oracle noise floor {fd:.3e} / {fr:.3e}")
        assert rdiff < br, (iters, rdiff, br)
        assert d < bd, (iters, d, bd)


@pytest.mark.parametrize("name", list(SYSTEMS))
@pytest.mark.parametrize("prec", [eofa.FP64, eofa.FP32, eofa.FP16S])
def test_cg_converged(c1ctx, name, prec):
    act, U, phi, out = oracle_c1(name)
    psi = torch.zeros(c1ctx.full_shape(1), dtype=torch.complex128, device="cuda")
    prm = eofa.make_params(tol=1e-10, inner_prec=prec)
    rc, st = c1ctx.eofa_cg_solve([SYSTEMS[name]], dev(phi[None]), psi, prm)
    assert rc == eofa.EOFA_OK, st
    assert st[0]["true_resid"] <= 1e-10 and st[0]["converged"] == 1
    got = host(psi)[0]
    # the oracle re-measures the residual of (H + beta Delta P) psi = phi
    res = np.sqrt(norm2(H_system(act, U, SYSTEMS[name], got) - phi) / norm2(phi))
    assert res <= 1.05e-10, res
    assert abs(res - st[0]["true_resid"]) < 1e-11
    assert rel2(got, out["psi"]) < 1e-7


@pytest.mark.parametrize("prec", [eofa.FP16S, eofa.FP32])
def test_wide_range_source(c1ctx, prec):
    """A source whose 5D sites are scaled by 10^u, u uniform in [-20, 30]
    (entries up to ~1e30, 50 orders of magnitude between sites): FP16 values
    with one FP32 scale per site hold every site in range (the FP32 inner
    solution and the FP64 outer loop too), and the shifted system still
    reaches an FP64 true residual of 1e-10, re-measured by the oracle."""
    act, U, phi, _ = oracle_c1("chi2")
    rng = np.random.default_rng(2300)
    scale = 10.0 ** rng.uniform(-20.0, 30.0, size=phi.shape[:-2])
    src = phi * scale[..., None, None]
    psi = torch.zeros(c1ctx.full_shape(1), dtype=torch.complex128, device="cuda")
    rc, st = c1ctx.eofa_cg_solve([SYSTEMS["chi2"]], dev(src[None]), psi,
                                 eofa.make_params(tol=1e-10, inner_prec=prec))
    assert rc == eofa.EOFA_OK and st[0]["converged"] == 1, st
    got = host(psi)[0]
    assert np.all(np.isfinite(got)) and np.abs(got).max() > 1e28
    res = np.sqrt(norm2(H_system(act, U, SYSTEMS["chi2"], got) - src) / norm2(src))
    assert res <= 1.05e-10, res


def test_cg_batched_equals_single(c1ctx):
    """Three different systems in one batched solve = three single solves."""
    names = list(SYSTEMS)
    act, U, phi, _ = oracle_c1(names[0])
    phis = np.stack([phi, synth.fermion(act.dims, act.Ls, seed=2001), synth.fermion(act.dims, act.Ls, seed=2002)])
    sysl = [SYSTEMS[n] for n in names]
    prm = eofa.make_params(fixed_iters=40)
    psi = torch.zeros(c1ctx.full_shape(3), dtype=torch.complex128, device="cuda")
    c1ctx.eofa_cg_solve(sysl, dev(phis), psi, prm)
    batched = host(psi)
    for r in range(3):
        one = torch.zeros(c1ctx.full_shape(1), dtype=torch.complex128, device="cuda")
        c1ctx.eofa_cg_solve([sysl[r]], dev(phis[r:r + 1]), one, prm)
        assert rel2(batched[r], host(one)[0]) < 1e-14


HB_ALPHA, HB_BETA = [0.35, 0.2, 0.9], [0.05, 2.0]
_HB = {}


def oracle_heatbath():
    """eqn eofa_heatbath by the oracle (mirror-mode solves at 1e-12) for
    HB_ALPHA, HB_BETA and eta (seed 2100) at the small workload."""
    if "phi" not in _HB:
        act, U, _, _ = oracle_c1("chi1")
        eta = synth.fermion(act.dims, act.Ls, seed=2100)

        def solve(sys_, rhs):
            return eo.solve_mirror(act, U, sys_, rhs, tol=1e-12)["psi"]

        _HB["eta"] = eta
        _HB["phi"] = oaction.heatbath(act, M1, M2, HB_ALPHA, HB_BETA, eta, solve)
    return _HB["eta"], _HB["phi"]


@pytest.mark.parametrize("use_guess", [0, 1])
def test_heatbath_matches_oracle(c1ctx, use_guess):
    """eqn eofa_heatbath on the GPU vs the oracle formula at the same alpha,
    beta and eta: all 2 N_p systems batched (use_guess = 0), or the poles of
    each side in sequence from chronological forecasts (Sec. VI B)."""
    eta, ref = oracle_heatbath()
    phi = torch.zeros(c1ctx.full_shape(1), dtype=torch.complex128, device="cuda")
    prm = eofa.make_params(tol=1e-11, use_guess=use_guess)
    rc, st = c1ctx.eofa_heatbath_solve(M1, M2, HB_ALPHA, HB_BETA, dev(eta[None]), phi, prm)
    assert rc == eofa.EOFA_OK
    assert all(s["converged"] for s in st)
    assert rel2(host(phi)[0], ref) < 1e-9


def test_heatbath_forecast_and_pole_tol(c1ctx):
    """Sec. VI B: poles solved one after another from chronological forecasts
    need fewer iterations than the batched solve (the first pole of each side
    has no forecast), and per-pole tolerances are met: every pole solution
    from eofa_heatbath_poles is re-measured by the oracle on the H form of its
    system, (H(m_op) + beta Delta_chi P_chi) y = Omega P eta."""
    act, U, _, _ = oracle_c1("chi1")
    eta_h = synth.fermion(act.dims, act.Ls, seed=2101)
    eta = dev(eta_h[None])
    beta = [0.01, 0.1, 0.5, 2.0]
    n = len(beta)
    sol_b = torch.zeros(c1ctx.full_shape(2 * n), dtype=torch.complex128, device="cuda")
    rc, st_b = c1ctx.eofa_heatbath_poles(M1, M2, beta, eta, sol_b, eofa.make_params(tol=1e-11))
    assert rc == eofa.EOFA_OK
    sol_f = torch.zeros_like(sol_b)
    rc, st_f = c1ctx.eofa_heatbath_poles(M1, M2, beta, eta, sol_f, eofa.make_params(tol=1e-11, use_guess=1))
    assert rc == eofa.EOFA_OK and all(s["converged"] for s in st_f)
    it_b, it_f = [s["iters"] for s in st_b], [s["iters"] for s in st_f]
    print("heatbath iterations per pole: batched", it_b, "forecast", it_f)
    assert it_f[0] == it_b[0] and it_f[n] == it_b[n]
    assert sum(it_f) < sum(it_b)
    ptol = [1e-6, 1e-8, 1e-10, 1e-11, 1e-7, 1e-9, 1e-10, 1e-11]
    sol_t = torch.zeros_like(sol_b)
    rc, st_t = c1ctx.eofa_heatbath_poles(M1, M2, beta, eta, sol_t, eofa.make_params(tol=1e-11, use_guess=1),
                                         pole_tol=ptol)
    assert rc == eofa.EOFA_OK
    W = oaction._omega_ops(act)
    rhs = [W["Wm"](eta_h), W["Wp"](eta_h)]
    for sols, tols in ((host(sol_f), [1e-11] * (2 * n)), (host(sol_t), ptol)):
        for r in range(2 * n):
            l, side = r % n, r // n
            sys_ = oaction.heatbath_systems(M1, M2, beta[l])[side]
            res = np.sqrt(norm2(H_system(act, U, sys_, sols[r]) - rhs[side]) / norm2(rhs[side]))
            assert res <= 1.05 * tols[r], (r, res, tols[r])
    for s, t in zip(st_t, ptol):
        assert s["converged"] == 1 and s["true_resid"] <= t


def test_forecast_matches_oracle(c1ctx):
    """eofa_forecast against oracle.action.chronological_guess (Sec. VI B) on
    the same right-hand side and the same earlier fields (three random fields
    and one oracle solution of a neighbouring pole), for a heatbath system."""
    act, U, _, _ = oracle_c1("chi1")
    sys_ = oaction.heatbath_systems(M1, M2, 0.3)[0]
    eta = synth.fermion(act.dims, act.Ls, seed=2102)
    rhs = oaction._omega_ops(act)["Wm"](eta)
    prev = [synth.fermion(act.dims, act.Ls, seed=2110 + k) for k in range(3)]
    near = oaction.heatbath_systems(M1, M2, 0.25)[0]
    prev.append(eo.solve_mirror(act, U, near, rhs, tol=1e-10)["psi"])
    ref = oaction.chronological_guess(lambda x: H_system(act, U, sys_, x), rhs, prev)
    guess = torch.zeros(c1ctx.full_shape(1), dtype=torch.complex128, device="cuda")
    c1ctx.eofa_forecast(sys_, dev(rhs[None]), dev(np.stack(prev)), len(prev), guess)
    got = host(guess)[0]
    assert rel2(got, ref) < 1e-10, rel2(got, ref)
    # a guess from the neighbouring pole's solution is a good start
    res = np.sqrt(norm2(H_system(act, U, sys_, got) - rhs) / norm2(rhs))
    assert res < 0.2, res


# --- errors ----------------------------------------------------------------------

def test_error_paths(c1ctx):
    act, U, phi, _ = oracle_c1("chi1")
    psi = torch.zeros(c1ctx.full_shape(1), dtype=torch.complex128, device="cuda")
    ph = dev(phi[None])
    with pytest.raises(eofa.EofaError) as e:
        c1ctx.eofa_cg_solve([(1.0, 0.04, 1.0, -1.0, 3)], ph, psi, eofa.make_params())
    assert e.value.code == eofa.EOFA_ERR_INVALID
    rc, st = c1ctx.eofa_cg_solve([SYSTEMS["chi2"]], ph, psi, eofa.make_params(max_iter=5, max_outer=1))
    assert rc == eofa.EOFA_ERR_NOT_CONVERGED and st[0]["converged"] == 0 and st[0]["iters"] <= 5
    # Sherman-Morrison breakdown: beta with 1 + chi beta v.x = 0
    Ls = act.Ls
    A0 = fifth.mee_blocks(Ls, M5, act.c, act.d, 1.0)[0]
    k = fifth.k_eofa(Ls, act.c, act.d, M1, M2)
    x = np.linalg.solve(A0, fifth.u_vec(Ls, act.c, act.d, 1.0, 1))
    beta = -1.0 / (k * x[Ls - 1])
    rc, st = c1ctx.eofa_cg_solve([(1.0, M1, M2, beta, 1)], ph, psi, eofa.make_params())
    assert rc == eofa.EOFA_ERR_BREAKDOWN
    # NaN in the source
    bad = phi.copy()
    bad[0, 0, 0, 0, 0, 0, 0] = np.nan
    rc, st = c1ctx.eofa_cg_solve([SYSTEMS["chi1"]], dev(bad[None]), psi, eofa.make_params())
    assert rc in (eofa.EOFA_ERR_BREAKDOWN, eofa.EOFA_ERR_NOT_CONVERGED) and st[0]["converged"] == 0
