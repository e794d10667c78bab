"""eofa_cg_solve_noalloc (workspace in the library's fixed scratch array, no
device allocation) against eofa_cg_solve on the same inputs and parameters.

Two calls in a row through the C ABI, the second with a smaller input:
  1. 4^4 x Ls = 8, three systems (H(m1), H(m2) - Delta_+ P_+, the heatbath
     LH system), FP16S inner CG with FP64 defect correction to 1e-10, and the
     same systems in FP64 at a fixed 40 iterations;
  2. 4 x 4 x 2 x 4 x Ls = 8, one system, FP64 to 1e-10.
The same kernels run in the same order with the same launch shape, so the
results agree to rounding (the bar of the FP64 kernels, 1e-13); both are
re-measured by the oracle. A lattice whose workspace exceeds the scratch
array is rejected with EOFA_ERR_INVALID before any device work.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.dwf import Action, System, H_system
from oracle.lattice import norm2
from paper_1706_05843_amd import eofa, synth

pytestmark = pytest.mark.gpu

M5, B5, C5 = 1.8, 1.5, 0.5
M1, M2 = 0.04, 1.0


def _ctx(dims, Ls, seed):
    act = Action(dims, Ls, M5, B5, C5, (1, 1, 1, -1))
    U = synth.gauge_field(dims, 0.3, seed=seed)
    ctx = eofa.Context(eofa.make_action(dims, Ls, M5, B5, C5), torch.from_numpy(U).cuda())
    return act, U, ctx


def _both(ctx, systems, phis, **kw):
    ph = torch.from_numpy(np.ascontiguousarray(phis)).cuda()
    a, b = torch.zeros_like(ph), torch.zeros_like(ph)
    prm = eofa.make_params(waves=2, rhs_block=1, **kw)
    rc_a, st_a = ctx.eofa_cg_solve(systems, ph, a, prm)
    rc_b, st_b = ctx.eofa_cg_solve_noalloc(systems, ph, b, prm)
    torch.cuda.synchronize()
    return (rc_a, st_a, a.cpu().numpy()), (rc_b, st_b, b.cpu().numpy())


def _rel(a, b):
    return np.sqrt(norm2(a - b) / norm2(b))


def test_noalloc_matches_solve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    # call 1: three systems on 4^4 x Ls = 8
    act, U, ctx = _ctx((4, 4, 4, 4), 8, 1000)
    systems = [System(M1, M1, M2, 0.0, -1), System(M2, M1, M2, -1.0, +1), System(M1, M1, M2, -0.5, -1)]
    phis = synth.fermion(act.dims, act.Ls, seed=2400, nrhs=3)
    for kw in (dict(tol=1e-10, inner_prec=eofa.FP16S, ring_slots=8), dict(fixed_iters=40, ring_slots=-1)):
        (rc_a, st_a, a), (rc_b, st_b, b) = _both(ctx, systems, phis, **kw)
        print("call 1", kw, "eofa_cg_solve", rc_a, [s["iters"] for s in st_a], "noalloc", rc_b,
              [s["iters"] for s in st_b], "bitwise equal:", np.array_equal(a, b))
        assert rc_a == rc_b
        assert [s["iters"] for s in st_a] == [s["iters"] for s in st_b]
        for r in range(3):
            assert _rel(b[r], a[r]) < 1e-13, (kw, r, _rel(b[r], a[r]))
            if "tol" in kw:
                assert st_b[r]["converged"] == 1
                res = np.sqrt(norm2(H_system(act, U, systems[r], b[r]) - phis[r]) / norm2(phis[r]))
                assert res <= 1.05e-10, (r, res)
    ctx.close()
    # call 2: a smaller lattice, one system
    act2, U2, ctx2 = _ctx((4, 4, 2, 4), 8, 1001)
    sys2 = [System(M2, M1, M2, -1.0, +1)]
    phi2 = synth.fermion(act2.dims, act2.Ls, seed=2401, nrhs=1)
    (rc_a, st_a, a), (rc_b, st_b, b) = _both(ctx2, sys2, phi2, tol=1e-10)
    print("call 2: eofa_cg_solve", rc_a, st_a[0]["iters"], "noalloc", rc_b, st_b[0]["iters"],
          "bitwise equal:", np.array_equal(a, b))
    assert rc_a == rc_b == eofa.EOFA_OK and st_a[0]["iters"] == st_b[0]["iters"]
    assert _rel(b[0], a[0]) < 1e-13
    res = np.sqrt(norm2(H_system(act2, U2, sys2[0], b[0]) - phi2[0]) / norm2(phi2[0]))
    assert res <= 1.05e-10, res
    ctx2.close()


def test_noalloc_rejects_oversize():
    """16^4 x Ls = 16 needs far more than the scratch array: a clear error, nothing run."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dims, Ls = (16, 16, 16, 16), 16
    ctx = eofa.Context(eofa.make_action(dims, Ls, M5, B5, C5), torch.from_numpy(synth.unit_gauge(dims)).cuda())
    phi = torch.zeros(ctx.full_shape(1), dtype=torch.complex128, device="cuda")
    psi = torch.zeros_like(phi)
    with pytest.raises(eofa.EofaError) as e:
        ctx.eofa_cg_solve_noalloc([System(M1, M1, M2, 0.0, -1)], phi, psi, eofa.make_params())
    assert e.value.code == eofa.EOFA_ERR_INVALID and "MiB" in str(e.value)
    ctx.close()
