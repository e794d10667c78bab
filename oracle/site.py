"""One-site evaluations of the operators, for sampled checks on lattices too
large for the full-lattice oracle.

Test infrastructure only: see the package docstring.

Plain loops over the eight neighbours, written from the definitions
(eqn Ddwf, eqn eofa_dop_def, eqn generic_eofa_system); only the s-columns of
a site and its neighbours are touched.
"""
import numpy as np

from . import fifth
from .lattice import GAMMA, GAMMA5, ID4, P_PLUS, P_MINUS


def _nbr(dims, x, mu, sign):
    """Neighbour coordinates (x, y, z, t) of x in direction sign*mu and the
    boundary phase index crossing flag."""
    y = list(x)
    L = dims[mu]
    y[mu] = (x[mu] + sign) % L
    crossed = (x[mu] == L - 1) if sign > 0 else (x[mu] == 0)
    return tuple(y), crossed


def _col(psi, x):
    """s-column psi[:, t, z, y, x] -> [Ls, 4, 3]."""
    return psi[:, x[3], x[2], x[1], x[0]]


def _chiral_apply(Ap, Am, col):
    """(A col)_s = sum_s' Ap[s,s'] P_+ col_s' + Am[s,s'] P_- col_s' for a column [Ls, 4, 3]."""
    cp = np.einsum("ab,sbc->sac", P_PLUS, col)
    cm = np.einsum("ab,sbc->sac", P_MINUS, col)
    return np.einsum("rs,sac->rac", Ap, cp) + np.einsum("rs,sac->rac", Am, cm)


def hop_column(act, U, col_of, x, adjoint=False):
    """Dhop applied at site x to every s: col_of(y) returns the s-column at y."""
    sg = -1.0 if adjoint else 1.0
    out = np.zeros((act.Ls, 4, 3), dtype=np.complex128)
    for mu in range(4):
        y, cr = _nbr(act.dims, x, mu, +1)
        ph = act.bc[mu] if cr else 1.0
        Uf = U[mu][x[3], x[2], x[1], x[0]]
        f = ph * np.einsum("ab,sib->sia", Uf, col_of(y))
        out += np.einsum("ij,sja->sia", ID4 - sg * GAMMA[mu], f)
        y, cr = _nbr(act.dims, x, mu, -1)
        ph = act.bc[mu] if cr else 1.0
        Ub = U[mu][y[3], y[2], y[1], y[0]].conj().T
        b = ph * np.einsum("ab,sib->sia", Ub, col_of(y))
        out += np.einsum("ij,sja->sia", ID4 + sg * GAMMA[mu], b)
    return -0.5 * out


def dslash_column(act, U, m, psi, x):
    """(Dhop D~(m) psi)(x, :) -- the off-parity block of D_DWF at site x."""
    Dp = fifth.Dtilde(act.Ls, act.c, act.d, m, +1)
    Dm = fifth.Dtilde(act.Ls, act.c, act.d, m, -1)
    return hop_column(act, U, lambda y: _chiral_apply(Dp, Dm, _col(psi, y)), x)


def dslash_dag_column(act, U, m, psi, x):
    """(D~(m)^T Dhop^dag psi)(x, :) -- its adjoint."""
    Dp = fifth.Dtilde(act.Ls, act.c, act.d, m, +1)
    Dm = fifth.Dtilde(act.Ls, act.c, act.d, m, -1)
    h = hop_column(act, U, lambda y: _col(psi, y), x, adjoint=True)
    return _chiral_apply(Dp.T, Dm.T, h)


def eofa_residual_column(act, U, sys, psi, phi, x):
    """(H(m_op) + beta Delta_chi P_chi) psi - phi at site x, all s, with
    H = gamma_5 R5 (D_W + M_+ P_+ + M_- P_-) (App. A closed forms)."""
    Ls = act.Ls
    Mp = fifth.M_closed(Ls, act.c, act.d, sys.m_op, +1)
    Mm = fifth.M_closed(Ls, act.c, act.d, sys.m_op, -1)
    col = _col(psi, x)
    d_eofa = (4.0 - act.M5) * col + hop_column(act, U, lambda y: _col(psi, y), x) + _chiral_apply(Mp, Mm, col)
    h = np.einsum("ab,sbc->sac", GAMMA5, d_eofa[::-1])
    if sys.beta != 0.0:
        D = fifth.Delta(Ls, act.c, act.d, sys.m_a, sys.m_b, sys.chi)
        Z = np.zeros_like(D)
        h = h + sys.beta * (_chiral_apply(D, Z, col) if sys.chi > 0 else _chiral_apply(Z, D, col))
    return h - _col(phi, x)
