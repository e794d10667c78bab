"""Host-side checks of the C ABI that need no GPU.

* libeofa.so loads and exports every function include/eofa.h declares;
* the ctypes structs match the C layout (a gcc-compiled probe prints sizeof
  and offsetof);
* argument validation happens before any device call;
* the fifth-dimension matrices the library builds on the host (App. A /
  App. B.2, Sherman-Morrison) agree with the oracle's.
"""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import fifth
from paper_1706_05843_amd import eofa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eofa.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(eofa_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_header():
    L = eofa.lib()
    names = declared()
    assert "eofa_cg_solve" in names and "eofa_dslash" in names and "eofa_heatbath_solve" in names
    for n in names:
        assert hasattr(L, n), n


def test_struct_layout_matches_c():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "eofa.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(eofa_action), sizeof(eofa_system), sizeof(eofa_solver_params), sizeof(eofa_solver_stats));
  printf("%zu %zu %zu %zu %zu\n", offsetof(eofa_action, M5), offsetof(eofa_action, bc), offsetof(eofa_solver_params, inner_tol), offsetof(eofa_solver_stats, hop_ms), offsetof(eofa_solver_params, waves));
  printf("%zu %zu %zu\n", offsetof(eofa_solver_params, precond), offsetof(eofa_solver_params, net), offsetof(eofa_solver_stats, fell_back));
  printf("%zu %zu %zu %zu\n", offsetof(eofa_solver_params, use_guess), offsetof(eofa_solver_params, form), offsetof(eofa_solver_params, keep_direction), offsetof(eofa_solver_params, ring_slots));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "probe")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    sizes = list(map(int, out))
    assert sizes[:4] == [ctypes.sizeof(eofa.Action), ctypes.sizeof(eofa.System),
                         ctypes.sizeof(eofa.SolverParams), ctypes.sizeof(eofa.SolverStats)]
    assert sizes[4:] == [eofa.Action.M5.offset, eofa.Action.bc.offset,
                         eofa.SolverParams.inner_tol.offset, eofa.SolverStats.hop_ms.offset,
                         eofa.SolverParams.waves.offset, eofa.SolverParams.precond.offset,
                         eofa.SolverParams.net.offset, eofa.SolverStats.fell_back.offset,
                         eofa.SolverParams.use_guess.offset, eofa.SolverParams.form.offset,
                         eofa.SolverParams.keep_direction.offset, eofa.SolverParams.ring_slots.offset]


@pytest.mark.parametrize("bad", [
    dict(dims=(4, 4, 4, 3)), dict(dims=(4, 4, 0, 4)), dict(Ls=7), dict(Ls=0), dict(Ls=34),
    dict(b5=1.5, c5=0.7), dict(bc=(1, 1, 1, 2)),
    # Vh * Ls = 2^28 5D sites per parity: beyond the 32-bit byte offsets of the
    # FP16S gathers (the site indexing alone would still fit), also when G-parity
    # doubles x
    dict(dims=(64, 64, 64, 128), Ls=16), dict(dims=(64, 64, 64, 64), Ls=16, bc=(2, 1, 1, -1)),
])
def test_create_rejects_invalid_action(bad):
    kw = dict(dims=(4, 4, 4, 4), Ls=8, M5=1.8, b5=1.5, c5=0.5, bc=(1, 1, 1, -1))
    kw.update(bad)
    act = eofa.make_action(**kw)
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    rc = eofa.lib().eofa_create(ctypes.byref(act), dummy, None, ctypes.byref(h))
    assert rc == eofa.EOFA_ERR_INVALID
    assert len(eofa.lib().eofa_last_error()) > 0


def _oracle_mats(Ls, M5, b5, c5, sysd):
    c, d = fifth.mobius_cd(b5, c5)
    m_op, m_a, m_b, beta, chi = sysd
    Ap, Am = fifth.mee_blocks(Ls, M5, c, d, m_op, beta, chi, m_a, m_b)
    Dp, Dm = fifth.Dtilde(Ls, c, d, m_op, +1), fifth.Dtilde(Ls, c, d, m_op, -1)
    Ip, Im = np.linalg.inv(Ap), np.linalg.inv(Am)
    Ep, Em = fifth.dense_blocks(Ls, M5, c, d, m_op, beta, chi, m_a, m_b)
    return {
        "mee": (Ap, Am), "mee_inv": (Ip, Im), "mee_t": (Ap.T, Am.T), "mee_inv_t": (Ip.T, Im.T),
        "mee_inv_t_dt_t": (Ip.T @ Dp.T, Im.T @ Dm.T), "neg_dt_t": (-Dp.T, -Dm.T),
        "dt_t": (Dp.T, Dm.T), "dt": (Dp, Dm),
        "dt_inv": (fifth.Dtilde_inv_closed(Ls, c, d, m_op, +1), fifth.Dtilde_inv_closed(Ls, c, d, m_op, -1)),
        # dense form from the App. A closed forms, not from M_ee D~^-1 as the library builds it
        "dee": (Ep, Em), "dee_inv": (np.linalg.inv(Ep), np.linalg.inv(Em)), "dee_t": (Ep.T, Em.T),
        "dee_inv_t": (np.linalg.inv(Ep).T, np.linalg.inv(Em).T),
    }


@pytest.mark.parametrize("Ls", [4, 8, 12, 16])
@pytest.mark.parametrize("sysd", [(0.04, 0.04, 1.0, 0.0, -1), (1.0, 0.04, 1.0, -1.0, 1),
                                  (0.04, 0.04, 1.0, -0.5, -1), (0.01, 0.01, 1.0, -0.3, 1)])
def test_fifth_matrices_match_oracle(Ls, sysd):
    act = eofa.make_action((4, 4, 4, 4), Ls, 1.8, 1.5, 0.5)
    ref = _oracle_mats(Ls, 1.8, 1.5, 0.5, sysd)
    for name in eofa.MAT_NAMES:
        got = eofa.eofa_fifth_matrix(act, sysd, name)
        for ch in range(2):
            scale = max(1.0, np.abs(ref[name][ch]).max())
            assert np.abs(got[ch] - ref[name][ch]).max() < 1e-13 * scale, (name, ch)


def test_fifth_matrix_breakdown():
    """beta chosen so that 1 + chi beta v.x = 0: Sherman-Morrison breaks down."""
    Ls, M5, b5, c5 = 8, 1.8, 1.5, 0.5
    c, d = fifth.mobius_cd(b5, c5)
    m_op, m_a, m_b, chi = 1.0, 0.04, 1.0, 1
    A0 = fifth.mee_blocks(Ls, M5, c, d, m_op)[0]
    k = fifth.k_eofa(Ls, c, d, m_a, m_b)
    x = np.linalg.solve(A0, fifth.u_vec(Ls, c, d, m_op, chi))
    beta = -1.0 / (chi * k * x[Ls - 1])
    act = eofa.make_action((4, 4, 4, 4), Ls, M5, b5, c5)
    with pytest.raises(eofa.EofaError) as e:
        eofa.eofa_fifth_matrix(act, (m_op, m_a, m_b, beta, chi), "mee_inv")
    assert e.value.code == eofa.EOFA_ERR_BREAKDOWN


def test_network_rejects_bad_channels():
    """Channel lists must run 1 -> ... -> 1 with 1..8 channels (checked before any device call)."""
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    for chans in ([1, 9, 1], [2, 4, 1], [1, 4, 2], [1]):
        arr = (ctypes.c_int32 * len(chans))(*chans)
        rc = eofa.lib().eofa_net_create(dummy, len(chans) - 1, arr, 0, 1.0, ctypes.byref(h))
        assert rc == eofa.EOFA_ERR_INVALID, chans


def test_pairs_and_solver_params_validation():
    dummy = ctypes.c_void_p(16)
    rec, its = ctypes.c_int32(), ctypes.c_int32()
    sysl = eofa.make_systems([(0.1, 0.0, 0.0, 0.0, 1)])
    rc = eofa.lib().eofa_cg_pairs(dummy, sysl, dummy, 0, 0, 1, 1e-8, 10, dummy, dummy, ctypes.byref(rec),
                                  ctypes.byref(its), None)
    assert rc == eofa.EOFA_ERR_INVALID
    prm = eofa.make_params(precond=2)
    rc = eofa.lib().eofa_cg_solve(dummy, sysl, dummy, ctypes.c_void_p(32), 1, ctypes.byref(prm), None, None)
    assert rc == eofa.EOFA_ERR_INVALID
    prm = eofa.make_params(precond=1, fixed_iters=5)
    rc = eofa.lib().eofa_cg_solve(dummy, sysl, dummy, ctypes.c_void_p(32), 1, ctypes.byref(prm), None, None)
    assert rc == eofa.EOFA_ERR_INVALID

    for kw in (dict(form=2), dict(form=1, precond=1), dict(ring_slots=3), dict(ring_slots=32),
               dict(ring_slots=-2), dict(ring_slots=16, check_every=8), dict(waves=3), dict(waves=8),
               dict(rhs_block=-1)):
        prm = eofa.make_params(**kw)
        rc = eofa.lib().eofa_cg_solve(dummy, sysl, dummy, ctypes.c_void_p(32), 1, ctypes.byref(prm), None, None)
        assert rc == eofa.EOFA_ERR_INVALID, kw
    # heatbath and force take the Cayley form only
    prm = eofa.make_params(form=1)
    a = (ctypes.c_double * 1)(1.0)
    rc = eofa.lib().eofa_heatbath_solve(dummy, ctypes.c_double(0.1), ctypes.c_double(1.0), 1, a, a, None, dummy,
                                        ctypes.c_void_p(32), ctypes.byref(prm), None, None)
    assert rc == eofa.EOFA_ERR_INVALID
    rc = eofa.lib().eofa_force(dummy, ctypes.c_double(0.1), ctypes.c_double(1.0), dummy, ctypes.c_void_p(32),
                               ctypes.byref(prm), None, None)
    assert rc == eofa.EOFA_ERR_INVALID
    rc = eofa.lib().eofa_heatbath_poles(dummy, ctypes.c_double(0.1), ctypes.c_double(1.0), 1, a, None, dummy,
                                        ctypes.c_void_p(32), ctypes.byref(prm), None, None)
    assert rc == eofa.EOFA_ERR_INVALID
    # chronological forecast: 1..32 earlier solutions
    for n_prev in (0, 33):
        rc = eofa.lib().eofa_forecast(dummy, sysl, dummy, ctypes.c_void_p(64), n_prev, ctypes.c_void_p(32), None)
        assert rc == eofa.EOFA_ERR_INVALID, n_prev
