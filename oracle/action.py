"""The EOFA action operator and heatbath.

Test infrastructure only: see the package docstring.

* eqn eofa_action:
    M_EOFA = 1 - k P_- Omega_-^dag H(m1)^-1 Omega_- P_-
               + k P_+ Omega_+^dag [H(m2) - Delta_+(m1, m2) P_+]^-1 Omega_+ P_+
* eqn eofa_heatbath (Woodbury form of a rational f(M_EOFA) with
  f(x) = alpha_0 + sum_l alpha_l / (beta_l + x), gamma_l = 1/(1 + beta_l)):
    phi = alpha_0 eta + sum_l alpha_l gamma_l { eta
            + k gamma_l P_- Omega_-^dag [H(m1) - gamma_l Delta_-(m1,m2) P_-]^-1 Omega_- P_- eta
            - k gamma_l P_+ Omega_+^dag [H(m2) - beta_l gamma_l Delta_+(m1,m2) P_+]^-1 Omega_+ P_+ eta }
  Reading: the printed sum runs over "k = 1..N_p" but its terms carry the
  index l; l is the pole index and k stays the EOFA constant of App. A.
* eqn heatbath_rel_err: eps = |eta^dag eta - phi^dag M_EOFA phi| / eta^dag eta
  (pinned against the dense eigendecomposition of M_EOFA on 2^4 x Ls=4:
  zero for phi = M_EOFA^(-1/2) eta, the eigenbasis closed form for
  phi = f(M_EOFA) eta).

``solve(sys, rhs)`` is any solver of eqn generic_eofa_system (dense LU,
mirror mode or full CGNR) so the same formulas serve every route.
"""
import numpy as np

from . import fifth
from .dwf import System, apply_s
from .lattice import vdot


def _omega_ops(act):
    Om_p = fifth.Omega(act.Ls, act.c, act.d, +1)
    Om_m = fifth.Omega(act.Ls, act.c, act.d, -1)
    Z = np.zeros_like(Om_p)
    return dict(
        Wp=lambda x: apply_s(Om_p, Z, x),          # Omega_+ P_+
        Wm=lambda x: apply_s(Z, Om_m, x),          # Omega_- P_-
        Wp_adj=lambda x: apply_s(Om_p.T, Z, x),    # P_+ Omega_+^dag
        Wm_adj=lambda x: apply_s(Z, Om_m.T, x),    # P_- Omega_-^dag
    )


def chi_systems(m1, m2):
    """The two systems of the action and force: H(m1) and H(m2) - Delta_+(m1, m2) P_+."""
    return (System(m1, m1, m2, 0.0, -1), System(m2, m1, m2, -1.0, +1))


def apply_meofa(act, m1, m2, phi, solve):
    k = fifth.k_eofa(act.Ls, act.c, act.d, m1, m2)
    W = _omega_ops(act)
    s1, s2 = chi_systems(m1, m2)
    chi1 = solve(s1, W["Wm"](phi))
    chi2 = solve(s2, W["Wp"](phi))
    return phi - k * W["Wm_adj"](chi1) + k * W["Wp_adj"](chi2)


def heatbath_systems(m1, m2, beta_l):
    g = 1.0 / (1.0 + beta_l)
    lh = System(m1, m1, m2, -g, -1)
    rh = System(m2, m1, m2, -beta_l * g, +1)
    return lh, rh


def heatbath(act, m1, m2, alpha, beta_poles, eta, solve):
    """alpha = [alpha_0, alpha_1..alpha_Np], beta_poles = [beta_1..beta_Np]."""
    k = fifth.k_eofa(act.Ls, act.c, act.d, m1, m2)
    W = _omega_ops(act)
    phi = alpha[0] * eta
    for l, bl in enumerate(beta_poles):
        g = 1.0 / (1.0 + bl)
        lh, rh = heatbath_systems(m1, m2, bl)
        y_lh = solve(lh, W["Wm"](eta))
        y_rh = solve(rh, W["Wp"](eta))
        phi = phi + alpha[l + 1] * g * (eta + k * g * W["Wm_adj"](y_lh)
                                        - k * g * W["Wp_adj"](y_rh))
    return phi


def heatbath_error(act, m1, m2, eta, phi, solve):
    nn = vdot(eta, eta).real
    return abs(nn - vdot(phi, apply_meofa(act, m1, m2, phi, solve)).real) / nn


def chronological_guess(A, phi, psis):
    """Sec. VI B (after Brower et al.): the guess sum_k c_k psi_k minimising
    psi^dag A psi - phi^dag psi - psi^dag phi over the span of psis, from
    sum_k c_k psi_l^dag A psi_k = psi_l^dag phi (A an operator callable)."""
    N = len(psis)
    Apsi = [A(p) for p in psis]
    G = np.array([[vdot(psis[l], Apsi[k]) for k in range(N)] for l in range(N)])
    f = np.array([vdot(psis[l], phi) for l in range(N)])
    c = np.linalg.solve(G, f)
    return sum(ck * p for ck, p in zip(c, psis))

