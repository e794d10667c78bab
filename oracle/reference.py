"""Independent routes to the EOFA-system solution ("reference mode").

Test infrastructure only: see the package docstring.

None of these uses the even-odd split, the Cayley form or the rank-one
Sherman-Morrison algebra, so agreement with ``eo.solve_mirror`` checks those
steps of the paper's route.

* ``dense_matrix`` -- any field operator as an explicit matrix (apply it to
  every unit vector); solved by LU.
* ``solve_full_cgnr`` -- CG on the normal equations of
  H(m_op) + beta Delta_chi P_chi itself (eqn generic_eofa_system), with
  D_EOFA taken from the App. A closed forms of M_+-.
* ``solve_free_field`` -- U = 1: the Wilson operator is diagonal in momentum,
  D_W(p) = (4 - M5) - sum_mu cos p_mu + i sum_mu gamma_mu sin p_mu, with
  p_mu = (2 pi n + theta_mu)/L_mu, theta = 0 (periodic) or pi
  (antiperiodic); each momentum is a (4 Ls) x (4 Ls) solve.
"""
import numpy as np

from . import fifth
from .dwf import H_system
from .eo import cgnr
from .lattice import GAMMA, GAMMA5, P_PLUS, P_MINUS, ID4


def dense_matrix(op, field_shape, batch=256):
    n = int(np.prod(field_shape))
    M = np.zeros((n, n), dtype=np.complex128)
    for j0 in range(0, n, batch):
        j1 = min(n, j0 + batch)
        E = np.zeros((j1 - j0, n), dtype=np.complex128)
        E[np.arange(j1 - j0), np.arange(j0, j1)] = 1.0
        cols = op(E.reshape((j1 - j0,) + tuple(field_shape)))
        M[:, j0:j1] = cols.reshape(j1 - j0, n).T
    return M


def solve_dense(act, U, sys, phi):
    M = dense_matrix(lambda x: H_system(act, U, sys, x), act.field_shape)
    return np.linalg.solve(M, phi.ravel()).reshape(phi.shape)


def solve_full_cgnr(act, U, sys, phi, tol=1e-13, max_iter=100000):
    """The system matrix is Hermitian (H Hermitian, Delta_chi P_chi
    Hermitian), so its adjoint is itself."""
    op = lambda x: H_system(act, U, sys, x)
    x, n, _ = cgnr(op, op, phi, tol=tol, max_iter=max_iter)
    return x, n


def _momenta(L, bc):
    theta = np.pi if bc < 0 else 0.0
    return (2.0 * np.pi * np.arange(L) + theta) / L


def solve_free_field(act, sys, phi):
    """Free-field (U = 1) solution of eqn generic_eofa_system by FFT."""
    lx, ly, lz, lt = act.dims
    Ls, c, d = act.Ls, act.c, act.d
    Ls_ = Ls
    # twist so every direction becomes periodic: chi(x) = e^{-i theta x} psi(x)
    axes_len = (lt, lz, ly, lx)
    bcs = (act.bc[3], act.bc[2], act.bc[1], act.bc[0])
    mus = (3, 2, 1, 0)
    twist = np.ones(axes_len, dtype=np.complex128)
    for ax, (L, bc) in enumerate(zip(axes_len, bcs)):
        theta = np.pi / L if bc < 0 else 0.0
        shape = [1, 1, 1, 1]
        shape[ax] = L
        twist = twist * np.exp(-1j * theta * np.arange(L)).reshape(shape)
    chi = phi * twist[None, ..., None, None]
    chih = np.fft.fftn(chi, axes=(1, 2, 3, 4))

    Mp = fifth.M_closed(Ls, c, d, sys.m_op, +1)
    Mm = fifth.M_closed(Ls, c, d, sys.m_op, -1)
    R5 = fifth.R5(Ls)
    G5R5 = np.kron(R5, GAMMA5)
    base = np.kron(Mp, P_PLUS) + np.kron(Mm, P_MINUS)
    shift = 0.0
    if sys.beta != 0.0:
        D = fifth.Delta(Ls, c, d, sys.m_a, sys.m_b, sys.chi)
        shift = sys.beta * np.kron(D, P_PLUS if sys.chi > 0 else P_MINUS)
    moms = [_momenta(L, bc) for L, bc in zip(axes_len, bcs)]
    out = np.zeros_like(chih)
    for it in range(lt):
        for iz in range(lz):
            for iy in range(ly):
                for ix in range(lx):
                    p = {3: moms[0][it], 2: moms[1][iz], 1: moms[2][iy], 0: moms[3][ix]}
                    dw = (4.0 - act.M5) * ID4
                    for mu in range(4):
                        dw = dw - np.cos(p[mu]) * ID4 + 1j * np.sin(p[mu]) * GAMMA[mu]
                    A = G5R5 @ (np.kron(np.eye(Ls_), dw) + base) + shift
                    rhs = chih[:, it, iz, iy, ix].reshape(Ls * 4, 3)
                    out[:, it, iz, iy, ix] = np.linalg.solve(A, rhs).reshape(Ls, 4, 3)
    psi = np.fft.ifftn(out, axes=(1, 2, 3, 4)) / twist[None, ..., None, None]
    return psi
