"""Fifth-dimension (Ls x Ls, real) matrices of the Mobius EOFA operators.

Test infrastructure only: see the package docstring.

Parameters follow Sec. II: the Mobius weights are c and d with d = 1/2
fixed; the inputs b5, c5 map to c = (b5 + c5)/2, d = (b5 - c5)/2 (a
reading; b5 - c5 = 1 gives d = 1/2). Every matrix here acts on one
chirality: the "+" matrix multiplies P_+ psi, the "-" matrix P_- psi.

Sources:
* L_+-                            Sec. II, below eqn Ddwf
* D~ = d(1 - L) + c(1 + L)        eqn eofa_dop_def
* N(m) = (c+d)^Ls + m (c-d)^Ls    eqn dtilde_det (det D~ = N(m)^{12V})
* k, Omega_+-, Delta_+-, M_+-,
  D~^-1 closed forms              App. A (Mobius kernel)
* Shamir forms                    App. A (Shamir kernel)
* u_+-, v_+-                      App. B.2, eqn delta_rank_one
* R5                              Sec. II, (R5)_{ss'} = delta_{s, Ls-1-s'}
* dense same-site block           eqn eofa_dop_def with D_W -> (4 - M5), plus
                                  gamma_5 R5 times the shift of eqn
                                  generic_eofa_system
"""
import numpy as np


def mobius_cd(b5, c5):
    """(c, d) of the paper from the Mobius (b5, c5)."""
    return 0.5 * (b5 + c5), 0.5 * (b5 - c5)


def _sgn(n):
    """(-1)^n for any integer n."""
    return -1.0 if (n % 2) else 1.0


def L_plus(Ls, m):
    """(L_+)_{ss'} = delta_{s-1,s'} for 1 <= s <= Ls-1, -m delta_{Ls-1,s'} for s = 0."""
    A = np.zeros((Ls, Ls))
    for s in range(Ls):
        if s == 0:
            A[s, Ls - 1] = -m
        else:
            A[s, s - 1] = 1.0
    return A


def L_minus(Ls, m):
    """(L_-)_{ss'} = (L_+)_{s's}."""
    return L_plus(Ls, m).T.copy()


def R5(Ls):
    return np.eye(Ls)[::-1].copy()


def Dtilde(Ls, c, d, m, chir):
    """Chiral block of D~ = d(1 - L) + c(1 + L)."""
    L = L_plus(Ls, m) if chir > 0 else L_minus(Ls, m)
    return d * (np.eye(Ls) - L) + c * (np.eye(Ls) + L)


def N(Ls, c, d, m):
    return (c + d) ** Ls + m * (c - d) ** Ls


def k_eofa(Ls, c, d, m1, m2):
    """App. A, Mobius k."""
    return 2.0 * c * (m2 - m1) * (c + d) ** (2 * Ls) / (N(Ls, c, d, m1) * N(Ls, c, d, m2))


def Omega(Ls, c, d, chir):
    """App. A: Omega_+- is an Ls x Ls matrix whose only non-zero column is s' = 0."""
    A = np.zeros((Ls, Ls))
    for s in range(Ls):
        if chir > 0:
            A[s, 0] = _sgn(s + 1) * (c - d) ** (Ls - s - 1) / (c + d) ** (Ls - s)
        else:
            A[s, 0] = _sgn(s) * (c - d) ** s / (c + d) ** (s + 1)
    return A


def Delta(Ls, c, d, m1, m2, chir):
    """App. A, eqns mobius_Dp / mobius_Dm."""
    A = np.zeros((Ls, Ls))
    den = N(Ls, c, d, m1) * N(Ls, c, d, m2)
    for s in range(Ls):
        for t in range(Ls):
            if chir > 0:
                num = (c + d) ** (s + t) * (c - d) ** (2 * (Ls - 1) - s - t)
            else:
                num = (c + d) ** (2 * (Ls - 1) - s - t) * (c - d) ** (s + t)
            A[s, t] = _sgn(s + t) * 2.0 * c * (m2 - m1) * num / den
    return A


def M_closed(Ls, c, d, m, chir):
    """App. A, eqns mobius_Mp / mobius_Mm (dense in s)."""
    A = np.zeros((Ls, Ls))
    n = N(Ls, c, d, m)
    diag = ((c + d) ** (Ls - 1) - m * (c - d) ** (Ls - 1)) / n
    for s in range(Ls):
        for t in range(Ls):
            if s == t:
                A[s, t] = diag
            elif s > t:   # Theta_{s-s'-1}
                if chir > 0:
                    A[s, t] = _sgn(s - t) * 2 * c * (c + d) ** (Ls - s + t - 1) * (c - d) ** (s - t - 1) / n
                else:
                    A[s, t] = _sgn(t - s + 1) * 2 * c * m * (c + d) ** (s - t - 1) * (c - d) ** (Ls - s + t - 1) / n
            else:         # Theta_{s'-s-1}
                if chir > 0:
                    A[s, t] = _sgn(s - t + 1) * 2 * c * m * (c + d) ** (t - s - 1) * (c - d) ** (Ls + s - t - 1) / n
                else:
                    A[s, t] = _sgn(s - t) * 2 * c * (c + d) ** (Ls + s - t - 1) * (c - d) ** (t - s - 1) / n
    return A


def Dtilde_inv_closed(Ls, c, d, m, chir):
    """App. A closed form of D~(m)^-1, chiral block."""
    A = np.zeros((Ls, Ls))
    n = N(Ls, c, d, m)
    for s in range(Ls):
        for t in range(Ls):
            if chir > 0:
                v = m * _sgn(s - t + 1) * (c + d) ** (t - s - 1) * (c - d) ** (Ls + s - t) / n
                if s >= t:
                    v += _sgn(s - t) * (c - d) ** (s - t) / (c + d) ** (s - t + 1)
            else:
                v = m * _sgn(t - s + 1) * (c + d) ** (s - t - 1) * (c - d) ** (Ls + t - s) / n
                if t >= s:
                    v += _sgn(t - s) * (c - d) ** (t - s) / (c + d) ** (t - s + 1)
            A[s, t] = v
    return A


def shamir_forms(Ls, m1, m2, m, chir):
    """App. A Shamir kernel (c = d = 1/2): k, Omega, Delta, M(m).

    Reading: the printed Shamir M_+- place the mass corner at (Ls-1, 0) for
    M_+ and (0, Ls-1) for M_-, which is the transpose of what M = 1 - L
    (D~ = 1 for Shamir) gives and of the corners in App. B's Shamir
    same-parity block. The corners here follow M = 1 - L.
    """
    k = m2 - m1
    Om = np.zeros((Ls, Ls))
    De = np.zeros((Ls, Ls))
    M = np.eye(Ls)
    if chir > 0:
        Om[Ls - 1, 0] = 1.0
        De[Ls - 1, Ls - 1] = m2 - m1
        for s in range(1, Ls):
            M[s, s - 1] = -1.0
        M[0, Ls - 1] = m
    else:
        Om[0, 0] = 1.0
        De[0, 0] = m2 - m1
        for s in range(Ls - 1):
            M[s, s + 1] = -1.0
        M[Ls - 1, 0] = m
    return k, Om, De, M


def u_vec(Ls, c, d, m_op, chir):
    """App. B.2: u_+- of the rank-one form Delta~ = u (x) v; N taken at the operator mass."""
    n = N(Ls, c, d, m_op)
    u = np.zeros(Ls)
    for s in range(Ls):
        if chir > 0:
            u[s] = _sgn(s) * (c - d) ** s / (c + d) ** (Ls + s + 1) * n
        else:
            u[s] = _sgn(s + 1) * (c - d) ** (Ls - 1 - s) / (c + d) ** (2 * Ls - s) * n
    return u


def v_vec(Ls, k, chir):
    v = np.zeros(Ls)
    v[Ls - 1 if chir > 0 else 0] = k
    return v


def Delta_tilde(Ls, c, d, m_op, m_a, m_b, chir):
    """Delta~_+- = R5 Delta_+-(m_a, m_b) D~_+-(m_op)  (App. B.2), as a matrix product."""
    return R5(Ls) @ Delta(Ls, c, d, m_a, m_b, chir) @ Dtilde(Ls, c, d, m_op, chir)


def mee_blocks(Ls, M5, c, d, m_op, beta=0.0, chi=0, m_a=0.0, m_b=0.0):
    """Same-parity block of the Cayley-form system, per chirality.

    The site-local part of D_DWF(m) (eqn Ddwf with D_W -> (4 - M5)) is
    ((c+d)(4-M5) + 1) 1 + ((c-d)(4-M5) - 1) L; the preconditioned EOFA
    system (eqn precond_mobius_eofa_system) adds +- beta Delta~_+- on the
    P_+- block of chirality chi.
    """
    out = []
    for chir in (+1, -1):
        L = L_plus(Ls, m_op) if chir > 0 else L_minus(Ls, m_op)
        A = ((c + d) * (4 - M5) + 1) * np.eye(Ls) + ((c - d) * (4 - M5) - 1) * L
        if beta != 0.0 and chi == chir:
            A = A + chir * beta * Delta_tilde(Ls, c, d, m_op, m_a, m_b, chir)
        out.append(A)
    return out[0], out[1]


def sherman_morrison_inverse(A0, sigma, u, v):
    """(A0 + sigma u v^T)^-1 = A0^-1 - sigma A0^-1 u v^T A0^-1 / (1 + sigma v^T A0^-1 u)
    (eqn sherman_morrison_mobius_inv in its generic form), A0^-1 by LU."""
    A0i = np.linalg.inv(A0)
    x = A0i @ u
    den = 1.0 + sigma * (v @ x)
    if den == 0.0:
        raise ZeroDivisionError("Sherman-Morrison denominator vanishes")
    return A0i - sigma * np.outer(x, v @ A0i) / den


def dense_blocks(Ls, M5, c, d, m_op, beta=0.0, chi=0, m_a=0.0, m_b=0.0):
    """Same-site block of gamma_5 R5 (H(m_op) + beta Delta_chi P_chi), per chirality.

    gamma_5 R5 H = D_EOFA (Sec. II); its site-local part is (4 - M5) 1 + M_+-
    (eqn eofa_dop_def, App. A closed forms). gamma_5 R5 beta Delta_chi P_chi
    acts on chirality chi as chi beta R5 Delta_chi (gamma_5 = chi there).
    Dense in s: the system without the Cayley-form preconditioning.
    """
    out = []
    for chir in (+1, -1):
        A = (4.0 - M5) * np.eye(Ls) + M_closed(Ls, c, d, m_op, chir)
        if beta != 0.0 and chi == chir:
            A = A + chir * beta * R5(Ls) @ Delta(Ls, c, d, m_a, m_b, chir)
        out.append(A)
    return out[0], out[1]
