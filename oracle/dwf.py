"""5D Mobius domain-wall operators on full (both-parity) lattices.

Test infrastructure only: see the package docstring.

Field shape: [..., Ls, T, Z, Y, X, 4, 3]; the s axis is axis -7.

* D_DWF (eqn Ddwf):
    D_DWF = ((c+d) D_W + 1) delta_{ss'} + ((c-d) D_W - 1) L_{ss'}
  with D_W acting after L in the second term.
* D_EOFA (eqn eofa_dop_def): D_W delta_{ss'} + M_+ P_+ + M_- P_-.
* H = gamma_5 R5 D_EOFA (Sec. II).
* the EOFA system (eqn generic_eofa_system):
    (H(m_op) + beta Delta_chi(m_a, m_b) P_chi) psi = phi.
* its non-Hermitian form gamma_5 R5 (H + beta Delta P) = D_EOFA +
  gamma_5 R5 beta Delta P (dense_op), the matrix the Cayley form
  right-preconditions with D~^-1 (App. B.2).
"""
import numpy as np

from . import fifth
from .lattice import wilson, chiral, gamma5

S_AXIS = -7


class Action:
    """Mobius action parameters: dims = (Lx, Ly, Lz, Lt), Ls, M5, b5, c5, bc[4]."""

    def __init__(self, dims, Ls, M5, b5, c5, bc=(1, 1, 1, -1)):
        self.dims = tuple(int(v) for v in dims)
        self.Ls = int(Ls)
        self.M5 = float(M5)
        self.c, self.d = fifth.mobius_cd(b5, c5)
        self.bc = tuple(float(v) for v in bc)

    @property
    def field_shape(self):
        """G-parity in x (bc[0] == 2): flavour-doubled, flavour axis first."""
        lx, ly, lz, lt = self.dims
        shape = (self.Ls, lt, lz, ly, lx, 4, 3)
        return (2,) + shape if self.bc[0] == 2 else shape


def apply_s(Ap, Am, psi):
    """(A psi)_s = sum_s' Ap[s,s'] P_+ psi_s' + Am[s,s'] P_- psi_s'."""
    def mat(A, f):
        g = np.tensordot(A, np.moveaxis(f, S_AXIS, 0), axes=(1, 0))
        return np.moveaxis(g, 0, S_AXIS)
    return mat(Ap, chiral(psi, +1)) + mat(Am, chiral(psi, -1))


def L_op(act, m, psi, transpose=False):
    Lp, Lm = fifth.L_plus(act.Ls, m), fifth.L_minus(act.Ls, m)
    if transpose:
        Lp, Lm = Lp.T, Lm.T
    return apply_s(Lp, Lm, psi)


def Dtilde_op(act, m, psi, transpose=False):
    Dp = fifth.Dtilde(act.Ls, act.c, act.d, m, +1)
    Dm = fifth.Dtilde(act.Ls, act.c, act.d, m, -1)
    if transpose:
        Dp, Dm = Dp.T, Dm.T
    return apply_s(Dp, Dm, psi)


def R5_op(psi):
    return np.flip(psi, axis=S_AXIS)


def g5R5(psi):
    return gamma5(R5_op(psi))


def D_dwf(act, U, m, psi):
    """eqn Ddwf, written term by term."""
    c, d = act.c, act.d
    Lpsi = L_op(act, m, psi)
    return ((c + d) * wilson(U, psi, act.M5, act.bc) + psi
            + (c - d) * wilson(U, Lpsi, act.M5, act.bc) - Lpsi)


def D_dwf_adj(act, U, m, psi):
    """Adjoint of eqn Ddwf: ((c+d) D_W^dag + 1) + L^dag ((c-d) D_W^dag - 1)."""
    c, d = act.c, act.d
    Wd = wilson(U, psi, act.M5, act.bc, adjoint=True)
    return (c + d) * Wd + psi + L_op(act, m, (c - d) * Wd - psi, transpose=True)


def D_eofa(act, U, m, psi):
    """eqn eofa_dop_def with the App. A closed forms of M_+-(m)."""
    Mp = fifth.M_closed(act.Ls, act.c, act.d, m, +1)
    Mm = fifth.M_closed(act.Ls, act.c, act.d, m, -1)
    return wilson(U, psi, act.M5, act.bc) + apply_s(Mp, Mm, psi)


def shift_op(act, m_a, m_b, chi, psi):
    """Delta_chi(m_a, m_b) P_chi psi (App. A closed form of Delta)."""
    D = fifth.Delta(act.Ls, act.c, act.d, m_a, m_b, chi)
    Z = np.zeros_like(D)
    return apply_s(D, Z, psi) if chi > 0 else apply_s(Z, D, psi)


def H_system(act, U, sys, psi):
    """(H(m_op) + beta Delta_chi(m_a, m_b) P_chi) psi  (eqn generic_eofa_system)."""
    out = g5R5(D_eofa(act, U, sys.m_op, psi))
    if sys.beta != 0.0:
        out = out + sys.beta * shift_op(act, sys.m_a, sys.m_b, sys.chi, psi)
    return out


def dense_op(act, U, sys, psi):
    """(D_EOFA(m_op) + gamma_5 R5 beta Delta_chi P_chi) psi = gamma_5 R5 (H + beta Delta P) psi."""
    out = D_eofa(act, U, sys.m_op, psi)
    if sys.beta != 0.0:
        out = out + sys.beta * gamma5(R5_op(shift_op(act, sys.m_a, sys.m_b, sys.chi, psi)))
    return out


class System:
    """One EOFA linear system (eqn generic_eofa_system):
    (H(m_op) + beta Delta_chi(m_a, m_b) P_chi) psi = phi."""

    def __init__(self, m_op, m_a=0.0, m_b=0.0, beta=0.0, chi=1):
        self.m_op, self.m_a, self.m_b = float(m_op), float(m_a), float(m_b)
        self.beta, self.chi = float(beta), int(chi)


def cayley_op(act, U, sys, psi):
    """(D_DWF(m_op) + chi beta Delta~_chi) psi' (eqn precond_mobius_eofa_system)."""
    out = D_dwf(act, U, sys.m_op, psi)
    if sys.beta != 0.0:
        Dt = fifth.Delta_tilde(act.Ls, act.c, act.d, sys.m_op, sys.m_a, sys.m_b, sys.chi)
        Z = np.zeros_like(Dt)
        sh = apply_s(Dt, Z, psi) if sys.chi > 0 else apply_s(Z, Dt, psi)
        out = out + sys.chi * sys.beta * sh
    return out
