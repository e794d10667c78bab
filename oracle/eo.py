"""The paper's solve route for one EOFA system ("mirror mode").

Test infrastructure only: see the package docstring.

Steps, in the paper's order:
1. multiply the system by gamma_5 R5 (eqn non_hermit_sys): right-hand
   side b = gamma_5 R5 phi;
2. right-precondition with D~(m_op)^-1 (App. B.2, eqn
   precond_mobius_eofa_system): solve (D_DWF(m_op) + chi beta Delta~_chi)
   psi' = b, then psi = D~ psi';
3. even-odd Schur complement of that operator on the odd sublattice
   (App. B): (M_oo - M_oe M_ee^-1 M_eo) psi'_o = b_o - M_oe M_ee^-1 b_e;
   M_ee^-1 by Sherman-Morrison (eqn sherman_morrison_mobius_inv, generic
   form) on top of an LU inverse of the unshifted block;
4. CG on the normal equations (App. B: "CG applied to the normal
   equations") -- recurrences below;
5. psi'_e = M_ee^-1 (b_e - M_eo psi'_o), then psi = D~ psi'.

The off-parity blocks are the full-lattice D_DWF restricted to one parity
on input and the other on output; nothing is fused or reordered.
"""
import numpy as np

from . import fifth
from .dwf import apply_s, D_dwf, D_dwf_adj, Dtilde_op, g5R5, cayley_op, dense_op
from .lattice import restrict, norm2, hop

EVEN, ODD = 0, 1


class SchurSystem:
    def __init__(self, act, U, sys):
        self.act, self.U, self.sys = act, U, sys
        Ls, c, d = act.Ls, act.c, act.d
        self.Ap, self.Am = fifth.mee_blocks(Ls, act.M5, c, d, sys.m_op, sys.beta,
                                            sys.chi, sys.m_a, sys.m_b)
        # M_ee^-1: unshifted block by LU, shifted chirality by Sherman-Morrison
        A0p, A0m = fifth.mee_blocks(Ls, act.M5, c, d, sys.m_op)
        inv = {+1: np.linalg.inv(A0p), -1: np.linalg.inv(A0m)}
        if sys.beta != 0.0:
            A0 = A0p if sys.chi > 0 else A0m
            k = fifth.k_eofa(Ls, c, d, sys.m_a, sys.m_b)
            u = fifth.u_vec(Ls, c, d, sys.m_op, sys.chi)
            v = fifth.v_vec(Ls, k, sys.chi)
            inv[sys.chi] = fifth.sherman_morrison_inverse(A0, sys.chi * sys.beta, u, v)
        self.Ip, self.Im = inv[+1], inv[-1]

    # same-parity block and its inverse (site local, both parities alike)
    def mee(self, x):
        return apply_s(self.Ap, self.Am, x)

    def mee_adj(self, x):
        return apply_s(self.Ap.T, self.Am.T, x)

    def mee_inv(self, x):
        return apply_s(self.Ip, self.Im, x)

    def mee_inv_adj(self, x):
        return apply_s(self.Ip.T, self.Im.T, x)

    # off-parity blocks of D_DWF(m_op) (the shift is site local: no part here)
    def hop_block(self, x, out_par):
        d = self.act.dims
        return restrict(D_dwf(self.act, self.U, self.sys.m_op, restrict(x, d, 1 - out_par)), d, out_par)

    def hop_block_adj(self, x, out_par):
        d = self.act.dims
        return restrict(D_dwf_adj(self.act, self.U, self.sys.m_op, restrict(x, d, 1 - out_par)), d, out_par)

    def mhat(self, x):
        """M^ x = M_oo x - M_oe M_ee^-1 M_eo x on odd sites."""
        t = self.mee_inv(self.hop_block(x, EVEN))
        return self.mee(x) - self.hop_block(t, ODD)

    def mhat_adj(self, y):
        """M^dag y = M_oo^dag y - M_eo^dag M_ee^-dag M_oe^dag y."""
        t = self.mee_inv_adj(self.hop_block_adj(y, EVEN))
        return self.mee_adj(y) - self.hop_block_adj(t, ODD)

    def schur_source(self, b):
        d = self.act.dims
        be, bo = restrict(b, d, EVEN), restrict(b, d, ODD)
        return bo - self.hop_block(self.mee_inv(be), ODD)

    def reconstruct(self, xo, b):
        d = self.act.dims
        be = restrict(b, d, EVEN)
        xe = self.mee_inv(be - self.hop_block(xo, EVEN))
        return xe + restrict(xo, d, ODD)


def cgnr(op, op_adj, rhs, iters=None, tol=1e-10, max_iter=100000):
    """CG on op^dag op x = op^dag rhs from x = 0.

    r = op^dag rhs, p = r; each step: w = op p, alpha = |r|^2/|w|^2,
    q = op^dag w, x += alpha p, r -= alpha q, beta = |r_new|^2/|r|^2,
    p = r + beta p. Stops after ``iters`` steps if given, else when
    |r| <= tol |op^dag rhs|.
    """
    x = np.zeros_like(rhs)
    r = op_adj(rhs)
    p = r.copy()
    rr = norm2(r)
    stop = tol * tol * rr
    hist = [rr]
    n = 0
    while True:
        if iters is not None and n >= iters:
            break
        if iters is None and (rr <= stop or n >= max_iter):
            break
        w = op(p)
        alpha = rr / norm2(w)
        q = op_adj(w)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = norm2(r)
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        hist.append(rr)
        n += 1
    return x, n, hist


def solve_mirror(act, U, sys, phi, iters=None, tol=1e-10):
    """EOFA system by the paper's route. Returns dict with psi (solution of
    eqn generic_eofa_system), psi_prime, iters, the CGNR history and the
    true residual |phi - (H + beta Delta P) psi| / |phi| measured in the
    Cayley form |b - (D_DWF + chi beta Delta~) psi'| / |b|."""
    S = SchurSystem(act, U, sys)
    b = g5R5(phi)
    bt = S.schur_source(b)
    xo, n, hist = cgnr(S.mhat, S.mhat_adj, bt, iters=iters, tol=tol)
    xp = S.reconstruct(xo, b)
    psi = Dtilde_op(act, sys.m_op, xp)
    res = np.sqrt(norm2(b - cayley_op(act, U, sys, xp)) / norm2(b))
    schur = np.sqrt(norm2(bt - S.mhat(xo)) / norm2(phi))
    return dict(psi=psi, psi_prime=xp, iters=n, hist=hist, true_resid=res,
                schur_resid=schur, schur_source=bt, x_odd=xo)


class DenseSchurSystem(SchurSystem):
    """Even-odd Schur complement of the non-Cayley form gamma_5 R5 (H + beta
    Delta P) (dense_op): off-parity blocks the Wilson hop alone, same-parity
    blocks D_ee = (4 - M5) + M_chi(m_op) (+ chi beta R5 Delta_chi), dense in s
    (App. A closed forms; the comparison route to App. B.2's preconditioned
    form). Inverses by LU."""

    def __init__(self, act, U, sys):
        self.act, self.U, self.sys = act, U, sys
        self.Ap, self.Am = fifth.dense_blocks(act.Ls, act.M5, act.c, act.d, sys.m_op, sys.beta,
                                              sys.chi, sys.m_a, sys.m_b)
        self.Ip, self.Im = np.linalg.inv(self.Ap), np.linalg.inv(self.Am)

    def hop_block(self, x, out_par):
        d = self.act.dims
        return restrict(hop(self.U, restrict(x, d, 1 - out_par), self.act.bc), d, out_par)

    def hop_block_adj(self, x, out_par):
        d = self.act.dims
        return restrict(hop(self.U, restrict(x, d, 1 - out_par), self.act.bc, adjoint=True), d, out_par)


def solve_dense_form(act, U, sys, phi, iters=None, tol=1e-10):
    """The EOFA system without Cayley preconditioning: b = gamma_5 R5 phi,
    odd Schur complement of dense_op, CGNR, psi_e = D_ee^-1 (b_e - Dhop psi_o).
    Returns psi, iters, history and |b - dense_op psi| / |b|."""
    S = DenseSchurSystem(act, U, sys)
    b = g5R5(phi)
    bt = S.schur_source(b)
    xo, n, hist = cgnr(S.mhat, S.mhat_adj, bt, iters=iters, tol=tol)
    psi = S.reconstruct(xo, b)
    res = np.sqrt(norm2(b - dense_op(act, U, sys, psi)) / norm2(b))
    return dict(psi=psi, iters=n, hist=hist, true_resid=res, schur_source=bt, x_odd=xo)
