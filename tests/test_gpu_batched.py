"""Batched multi-right-hand-side solves, HIP graph replay and launch shapes.

* graph replay of the inner CG iterations gives bit-identical results to the
  eager launches (several replays, with the outer defect-correction work and
  host synchronisations between them);
* the hop kernels' launch shape (waves and right-hand sides per work-group)
  changes only the order of the partial sums: results agree to 1e-13;
* a batch of systems with their own (m_op, beta, chi) equals the single
  solves (1e-14), also in mixed precision;
* the batched solution update (a ring of R = 4, 8 or 16 search directions,
  x updated every R/2 iterations) equals the per-iteration update: the CG
  iterates are the same, x sums the same increments in another grouping
  (1e-13 FP64; FP32 solution storage below FP64: 1e-6);
* a right-hand side that breaks down stops alone: the others in its
  work-groups are unaffected (1e-13).
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
SYS = [System(M1, M1, M2, 0.0, -1), System(M2, M1, M2, -1.0, +1), System(M1, M1, M2, -0.5, -1),
       System(M2, M1, M2, -0.2, +1)]


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    act = Action((4, 4, 4, 8), 8, M5, B5, C5, (1, 1, 1, -1))
    U = synth.gauge_field(act.dims, 0.3, seed=1010)
    phis = synth.fermion(act.dims, act.Ls, seed=2010, nrhs=len(SYS))
    ctx = eofa.Context(eofa.make_action(act.dims, act.Ls, M5, B5, C5), torch.from_numpy(U).cuda())
    return act, U, phis, ctx


def solve(ctx, systems, phis, **kw):
    ph = torch.from_numpy(np.ascontiguousarray(phis)).cuda()
    psi = torch.zeros_like(ph)
    rc, st = ctx.eofa_cg_solve(systems, ph, psi, eofa.make_params(**kw))
    torch.cuda.synchronize()
    return rc, st, psi.cpu().numpy()


def rel2(a, b):
    return np.sqrt(norm2(a - b) / norm2(b))


@pytest.mark.parametrize("prec", [eofa.FP64, eofa.FP16S])
def test_graph_replay_equals_eager(setup, prec):
    act, U, phis, ctx = setup
    kw = dict(tol=1e-10, inner_prec=prec, check_every=8)
    rc0, st0, eager = solve(ctx, SYS, phis, **kw)
    rc1, st1, graph = solve(ctx, SYS, phis, use_graph=1, **kw)
    assert rc0 == rc1 == eofa.EOFA_OK
    assert [s["iters"] for s in st0] == [s["iters"] for s in st1]
    assert np.array_equal(eager, graph)
    for r, s in enumerate(SYS):  # and they solve the systems
        res = np.sqrt(norm2(H_system(act, U, s, graph[r]) - phis[r]) / norm2(phis[r]))
        assert res <= 1.05e-10


def test_launch_shapes_agree(setup):
    act, U, phis, ctx = setup
    ref = solve(ctx, SYS, phis, fixed_iters=40, waves=2, rhs_block=4)[2]
    for waves, rb in ((1, 1), (4, 3), (2, 2), (1, 4)):
        got = solve(ctx, SYS, phis, fixed_iters=40, waves=waves, rhs_block=rb)[2]
        assert rel2(got, ref) < 1e-13, (waves, rb, rel2(got, ref))


@pytest.mark.parametrize("Ls", [8, 12, 16])
def test_fp16s_launch_shapes_agree(Ls):
    """The FP16S hop kernels (SU(3) products on the matrix cores: the generic
    form at Ls = 8 and 12, with idle lanes at 12, and the row form at 16)
    under every launch shape: waves per work-group and right-hand sides per
    work-group change only the order of the CG reductions, so a few fixed
    iterations agree to FP16 storage precision, while a lane, site or
    right-hand-side mix-up would differ at O(1)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dims = (4, 4, 2, 4)
    U = synth.gauge_field(dims, 0.3, seed=1020 + Ls)
    phis = synth.fermion(dims, Ls, seed=2020 + Ls, nrhs=len(SYS))
    ctx = eofa.Context(eofa.make_action(dims, Ls, M5, B5, C5), torch.from_numpy(U).cuda())
    kw = dict(fixed_iters=3, inner_prec=eofa.FP16S)
    ref = solve(ctx, SYS, phis, waves=2, rhs_block=4, **kw)[2]
    for waves, rb in ((1, 1), (4, 3), (2, 2), (1, 4)):
        got = solve(ctx, SYS, phis, waves=waves, rhs_block=rb, **kw)[2]
        for r in range(len(SYS)):
            assert rel2(got[r], ref[r]) < 1e-4, (waves, rb, r, rel2(got[r], ref[r]))
    ctx.close()


@pytest.mark.parametrize("prec", [eofa.FP64, eofa.FP32])
def test_batch_equals_single(setup, prec):
    act, U, phis, ctx = setup
    kw = dict(fixed_iters=30, inner_prec=prec, waves=2, rhs_block=2)
    batch = solve(ctx, SYS, phis, **kw)[2]
    for r in range(len(SYS)):
        one = solve(ctx, [SYS[r]], phis[r:r + 1], **kw)[2][0]
        assert rel2(batch[r], one) < 1e-14


@pytest.mark.parametrize("prec", [eofa.FP64, eofa.FP16S])
def test_ring_sizes_agree(setup, prec):
    act, U, phis, ctx = setup
    kw = dict(fixed_iters=37, inner_prec=prec)  # 37: a partial flush at the end
    ref = solve(ctx, SYS, phis, ring_slots=-1, **kw)[2]
    for R in (4, 8, 16):
        rc, st, got = solve(ctx, SYS, phis, ring_slots=R, **kw)
        assert rc in (eofa.EOFA_OK, eofa.EOFA_ERR_NOT_CONVERGED) and st[0]["iters"] == 37
        d = rel2(got, ref)
        assert d < (1e-13 if prec == eofa.FP64 else 1e-6), (R, d)


@pytest.mark.parametrize("prec", [eofa.FP32, eofa.FP16S])
def test_twelve_rhs_converged_ls12(prec):
    """The batched workload's shape at reduced volume: 12 right-hand sides
    (6 on H(m1), 6 on H(m2) - Delta_+(m1, m2) P_+, m1 = 0.01) at Ls = 12 (the
    any-Ls kernels), inner CG below FP64 on the HIP-graph path with the
    autotuned launch shape, FP64 defect correction to a true residual of 1e-10;
    every solution re-measured by the oracle on the H form of its system."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m1 = 0.01
    act = Action((4, 4, 4, 4), 12, M5, B5, C5, (1, 1, 1, -1))
    U = synth.gauge_field(act.dims, 0.5, seed=1011)
    systems = [System(m1, m1, M2, 0.0, -1)] * 6 + [System(M2, m1, M2, -1.0, +1)] * 6
    phis = synth.fermion(act.dims, act.Ls, seed=2011, nrhs=12)
    ctx = eofa.Context(eofa.make_action(act.dims, act.Ls, M5, B5, C5), torch.from_numpy(U).cuda())
    rc, st, got = solve(ctx, systems, phis, tol=1e-10, inner_prec=prec, use_graph=1, check_every=16)
    assert rc == eofa.EOFA_OK, st
    for r, s in enumerate(systems):
        assert st[r]["converged"] == 1 and st[r]["true_resid"] <= 1e-10
        res = np.sqrt(norm2(H_system(act, U, s, got[r]) - phis[r]) / norm2(phis[r]))
        assert res <= 1.05e-10, (r, res)
    ctx.close()


@pytest.mark.parametrize("graph", [0, 1])
def test_one_rhs_breaking_down_leaves_the_others_exact(setup, graph):
    """A right-hand side whose FP32 inner residual overflows (source entries
    scaled by 1e60: finite in FP64, infinite once converted to FP32) stops on
    its own halt flag inside work-groups it shares with two healthy ones
    (rhs_block = 3). The healthy ones take the same iterations and reach the
    same solutions as a batch without it, and solve their systems."""
    act, U, phis, ctx = setup
    systems = [SYS[0], SYS[1], SYS[2]]
    bad = phis[:3].copy()
    bad[1] = bad[1] * 1e60
    kw = dict(tol=1e-10, inner_prec=eofa.FP32, waves=2, use_graph=graph, max_outer=6)
    rc, st, got = solve(ctx, systems, bad, rhs_block=3, **kw)
    assert rc != eofa.EOFA_OK and st[1]["converged"] == 0
    rc2, st2, ref = solve(ctx, [SYS[0], SYS[2]], phis[[0, 2]], rhs_block=2, **kw)
    assert rc2 == eofa.EOFA_OK
    for k, r in ((0, 0), (2, 1)):
        assert st[k]["converged"] == 1 and st[k]["iters"] == st2[r]["iters"]
        assert rel2(got[k], ref[r]) < 1e-13
        res = np.sqrt(norm2(H_system(act, U, systems[k], got[k]) - phis[k]) / norm2(phis[k]))
        assert res <= 1.05e-10
