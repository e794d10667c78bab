"""The Ls = 16 row form of the hop kernels (all precisions): every exchange
along s is a DPP row rotation, M_ee^-1 and M_ee^-T are the structured inverse
(geometric series of rho L summed in four doublings plus the Sherman-Morrison
term), the dense blocks of the dense form run along cyclic diagonals.

* mirror mode in FP64: 40 fixed iterations equal the oracle's to 1e-12;
* mirror mode in FP32: 20 fixed CGNR iterations through K1..K4 against the
  oracle's 20 FP64 iterations, for a +chirality shift (chi2), a -chirality
  shift (beta = -0.5) and no shift (chi1): 1e-4 relative (FP32 rounding of
  every operator application, amplified over 20 CG steps; a wrong operator
  gives O(1));
* converged FP16S solves of the same three systems reach the FP64 true
  residual 1e-10, re-measured by the oracle on the H form;
* the dense form at Ls = 16, FP16S, converges to 1e-10 as well.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import eo
from oracle.dwf import Action, System, H_system
from oracle.lattice import norm2
from paper_1706_05843_amd import eofa, synth

pytestmark = pytest.mark.gpu

M5, B5, C5 = 1.8, 1.5, 0.5
SYSTEMS = [System(1.0, 0.04, 1.0, -1.0, +1), System(0.04, 0.04, 1.0, -0.5, -1), System(0.1)]


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dims, Ls = (4, 4, 4, 4), 16
    act = Action(dims, Ls, M5, B5, C5, (1, 1, 1, -1))
    U = synth.gauge_field(dims, 0.4, seed=101)
    ctx = eofa.Context(eofa.make_action(dims, Ls, M5, B5, C5), torch.from_numpy(U).cuda())
    phi = synth.fermion(dims, Ls, 102, nrhs=3)
    return act, U, ctx, phi


def _res(act, U, sysm, sol, phi):
    return np.sqrt(norm2(H_system(act, U, sysm, sol) - phi) / norm2(phi))


@pytest.mark.parametrize("k", range(3))
def test_mirror_fp64(setup, k):
    """FP64: the oracle's iterates to 1e-12, as for the generic form."""
    act, U, ctx, phi = setup
    ref = eo.solve_mirror(act, U, SYSTEMS[k], phi[k], iters=40)["psi"]
    ph = torch.from_numpy(phi[k:k + 1]).cuda()
    psi = torch.zeros_like(ph)
    ctx.eofa_cg_solve([SYSTEMS[k]], ph, psi, eofa.make_params(fixed_iters=40))
    got = psi.cpu().numpy()[0]
    assert np.sqrt(norm2(got - ref) / norm2(ref)) < 1e-12


@pytest.mark.parametrize("k", range(3))
def test_mirror_fp32(setup, k):
    act, U, ctx, phi = setup
    ref = eo.solve_mirror(act, U, SYSTEMS[k], phi[k], iters=20)["psi"]
    ph = torch.from_numpy(phi[k:k + 1]).cuda()
    psi = torch.zeros_like(ph)
    ctx.eofa_cg_solve([SYSTEMS[k]], ph, psi, eofa.make_params(fixed_iters=20, inner_prec=eofa.FP32))
    got = psi.cpu().numpy()[0]
    assert np.sqrt(norm2(got - ref) / norm2(ref)) < 1e-4


@pytest.mark.parametrize("form", [0, 1])
def test_fp16s_converged(setup, form):
    act, U, ctx, phi = setup
    ph = torch.from_numpy(phi).cuda()
    psi = torch.zeros_like(ph)
    rc, st = ctx.eofa_cg_solve(SYSTEMS, ph, psi, eofa.make_params(tol=1e-10, inner_prec=eofa.FP16S, form=form,
                                                                   keep_direction=1))
    assert rc == eofa.EOFA_OK
    sol = psi.cpu().numpy()
    for r, s in enumerate(SYSTEMS):
        assert st[r]["converged"] == 1
        assert _res(act, U, s, sol[r], phi[r]) < 1.05e-10
