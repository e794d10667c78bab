"""Pseudofermion force of the EOFA action (Sec. IV C, eqn eofa_force).

Test infrastructure only: see the package docstring.

Definitions (the paper's):
* su(3) basis T^a = i lambda^a / 2 with the Gell-Mann matrices lambda^a, so
  Tr(T^a T^b) = -1/2 delta^ab (the normalisation the paper states);
* the force component F^a_{x,mu} = d/ds S(e^{s T^a} U_mu(x)) at s = 0, with
  S = phi^dag M_EOFA phi (eqn eofa_action), and the force matrix
  F_{x,mu} = sum_a T^a F^a_{x,mu}.

Dhop is linear in the links: d/ds a^dag Dhop(e^{s X} U_mu(x)) b at s = 0 is
a^dag Dhop(U') b where U' has every link zero except X U_mu(x) at (x, mu).
The paper's formula (eqn eofa_force) writes F^a through such bilinears of
chi_1 = H(m1)^-1 Omega_- P_- phi and chi_2 = [H(m2) - Delta_+ P_+]^-1 Omega_+ P_+ phi
with the EOFA constant k; in this library's Dhop (overall -1/2, eqn Ddwf) the
paper's "k/2" prefactor of the bilinear is that -1/2.
"""
import numpy as np

from . import fifth
from .action import apply_meofa, chi_systems, _omega_ops
from .dwf import g5R5
from .lattice import hop, vdot


def gell_mann():
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


def generators():
    """T^a = i lambda^a / 2."""
    return 0.5j * gell_mann()


def _site(x):
    """(x, y, z, t) -> array index (t, z, y, x) of a [T, Z, Y, X] field."""
    return (x[3], x[2], x[1], x[0])


def dhop_derivative(U, a, b, bc, x, mu, X):
    """a^dag (d/ds Dhop(e^{s X} U_mu(x)) at s = 0) b for 5D fields a, b."""
    Up = np.zeros_like(U)
    Up[mu][_site(x)] = X @ U[mu][_site(x)]
    return vdot(a, hop(Up, b, bc))


def chis(act, m1, m2, phi, solve):
    W = _omega_ops(act)
    s1, s2 = chi_systems(m1, m2)
    return solve(s1, W["Wm"](phi)), solve(s2, W["Wp"](phi))


def force_formula(act, U, m1, m2, phi, solve, links):
    """F^a at the given links [(x, mu)] from eqn eofa_force:
    F^a = k (g5 R5 chi_1)^dag dDhop chi_1 - k (g5 R5 chi_2)^dag dDhop chi_2."""
    k = fifth.k_eofa(act.Ls, act.c, act.d, m1, m2)
    chi1, chi2 = chis(act, m1, m2, phi, solve)
    a1, a2 = g5R5(chi1), g5R5(chi2)
    T = generators()
    out = np.zeros((len(links), 8))
    for n, (x, mu) in enumerate(links):
        for a in range(8):
            v = k * (dhop_derivative(U, a1, chi1, act.bc, x, mu, T[a])
                     - dhop_derivative(U, a2, chi2, act.bc, x, mu, T[a]))
            out[n, a] = v.real
    return out


def action_value(act, U, m1, m2, phi, solve_for):
    """S = phi^dag M_EOFA(U) phi; solve_for(U) returns a solver for that field."""
    return vdot(phi, apply_meofa(act, m1, m2, phi, solve_for(U))).real


def force_fd(act, U, m1, m2, phi, solve_for, x, mu, a, h=1e-5):
    """Central difference of S along e^{s T^a} U_mu(x)."""
    T = generators()[a]
    w, v = np.linalg.eigh(-1j * T)  # T = i H, H Hermitian: e^{sT} = V e^{i s w} V^dag
    vals = []
    for sgn in (+1, -1):
        E = (v * np.exp(1j * sgn * h * w)) @ v.conj().T
        Us = U.copy()
        Us[mu][_site(x)] = E @ U[mu][_site(x)]
        vals.append(action_value(act, Us, m1, m2, phi, solve_for))
    return (vals[0] - vals[1]) / (2 * h)


def force_matrix(Fa):
    """sum_a T^a F^a for F^a [..., 8] -> [..., 3, 3]."""
    return np.einsum("...a,aij->...ij", Fa, generators())
