"""Geometry and the 4D Wilson operator (Sec. II, eqn Ddwf, second line).

Test infrastructure only: see the package docstring.

D_W(x, x') = (4 - M5) delta_{x,x'}
             - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) delta_{x+mu, x'}
                            + (1 + gamma_mu) U_mu(x')^dag delta_{x-mu, x'} ]

The hopping part (everything but the (4 - M5) diagonal) is ``hop``.
"""
import numpy as np

# --- gamma matrices: chiral basis (the paper does not fix a basis) ---------

_s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_z2 = np.zeros((2, 2), dtype=np.complex128)
_i2 = np.eye(2, dtype=np.complex128)


def _offdiag(a, b):
    return np.block([[_z2, a], [b, _z2]])


# gamma_mu for mu = x, y, z, t
GAMMA = np.stack([
    _offdiag(-1j * _s1, 1j * _s1),
    _offdiag(-1j * _s2, 1j * _s2),
    _offdiag(-1j * _s3, 1j * _s3),
    _offdiag(_i2, _i2),
])
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ID4 = np.eye(4, dtype=np.complex128)
P_PLUS = 0.5 * (ID4 + GAMMA5)     # chiral projectors P_+- = (1 +- gamma_5)/2
P_MINUS = 0.5 * (ID4 - GAMMA5)


# --- lattice geometry -------------------------------------------------------
# Fermion fields are [..., T, Z, Y, X, 4, 3]; one gauge direction is
# [T, Z, Y, X, 3, 3]. Both carry two internal axes after the four lattice
# axes, so direction mu lives on axis -3 - mu for either.

def axis_of(mu):
    return -3 - mu


def shift(f, mu, sign, bc=1.0):
    """g(x) = f(x + sign * mu_hat), periodic in the array; a value that comes
    across the lattice edge is multiplied by ``bc``."""
    ax = f.ndim + axis_of(mu)
    g = np.roll(f, -sign, axis=ax)
    if bc != 1.0:
        edge = f.shape[ax] - 1 if sign > 0 else 0
        idx = [slice(None)] * f.ndim
        idx[ax] = edge
        g[tuple(idx)] *= bc
    return g


def parity_mask(dims):
    """1 on odd sites ((x+y+z+t) odd), 0 on even; array [T, Z, Y, X]."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly),
                             np.arange(lx), indexing="ij")
    return ((x + y + z + t) % 2).astype(np.int64)


def restrict(psi, dims, parity):
    """Zero every site whose parity is not ``parity`` (0 even, 1 odd)."""
    m = (parity_mask(dims) == parity).astype(np.float64)
    return psi * m[..., None, None]


def dagger(u):
    return np.conj(np.swapaxes(u, -1, -2))


def _spin(mat, f):
    return np.einsum("st,...tc->...sc", mat, f)


def _colour(u, f):
    return np.einsum("...ab,...sb->...sa", u, f)


def hop(U, psi, bc, adjoint=False):
    """Hopping part of D_W on every 4D slice of ``psi``.

    Dhop psi(x) = -1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x + mu)
                                + (1 + g_mu) U_mu(x - mu)^dag psi(x - mu) ].
    The adjoint follows from conjugate-transposing each matrix element:
    it is the same sum with gamma_mu -> -gamma_mu.
    bc[0] == 2 selects G-parity in x (``hop_gparity``).
    """
    if bc[0] == 2:
        return hop_gparity(U, psi, bc, adjoint)
    sg = -1.0 if adjoint else 1.0
    out = np.zeros_like(psi)
    for mu in range(4):
        fwd = _colour(U[mu], shift(psi, mu, +1, bc[mu]))
        ub = dagger(shift(U[mu], mu, -1))          # U_mu(x - mu)^dag
        bwd = _colour(ub, shift(psi, mu, -1, bc[mu]))
        out += _spin(ID4 - sg * GAMMA[mu], fwd) + _spin(ID4 + sg * GAMMA[mu], bwd)
    return -0.5 * out


def hop_gparity(U, psi, bc, adjoint=False):
    """Dhop with G-parity boundary conditions in x (Sec. II mentions G-parity
    ensembles but gives no operator form; this one is a reading): flavour-doubled
    fields psi[f] (axis 0, f = 0, 1); flavour 0 hops with U, flavour 1 with
    conj(U); across the x edge the fields obey psi(x + L) = Tw psi(x) with
    Tw = [[0, 1], [-1, 0]] on (psi_0, psi_1) and the links U(x + L) = conj(U(x)).
    bc[1..3] are the ordinary phases of y, z, t. Fields are 5D,
    [..., 2, Ls, T, Z, Y, X, 4, 3]: the flavour axis is the eighth from the end."""
    sg = -1.0 if adjoint else 1.0
    Uf = [U, np.conj(U)]
    psi = np.moveaxis(psi, -8, 0)
    out = np.zeros_like(psi)
    L = psi.shape[-3]
    for f in range(2):
        for mu in range(4):
            if mu != 0:
                fwd = _colour(Uf[f][mu], shift(psi[f], mu, +1, bc[mu]))
                ub = dagger(shift(Uf[f][mu], mu, -1))
                bwd = _colour(ub, shift(psi[f], mu, -1, bc[mu]))
            else:
                ax = psi[f].ndim - 3
                # psi_f(x + 1); at x = L - 1: (Tw psi(0))_f = psi_1(0) (f = 0), -psi_0(0) (f = 1)
                nxt = np.roll(psi[f], -1, axis=ax)
                other = psi[1] if f == 0 else -psi[0]
                idx = [slice(None)] * nxt.ndim
                idx[ax] = L - 1
                src = [slice(None)] * nxt.ndim
                src[ax] = 0
                nxt[tuple(idx)] = other[tuple(src)]
                fwd = _colour(Uf[f][0], nxt)
                # psi_f(x - 1); at x = 0: (Tw^-1 psi(L - 1))_f = -psi_1(L - 1) (f = 0), psi_0(L - 1) (f = 1)
                prv = np.roll(psi[f], +1, axis=ax)
                other = -psi[1] if f == 0 else psi[0]
                idx[ax] = 0
                src[ax] = L - 1
                prv[tuple(idx)] = other[tuple(src)]
                # U_x(x - 1); at x = 0 the link U_x(-1) = conj_(1-f)(U_x(L - 1))
                ul = np.roll(Uf[f][0], +1, axis=Uf[f][0].ndim - 3)
                ul[..., 0, :, :] = Uf[1 - f][0][..., L - 1, :, :]
                bwd = _colour(dagger(ul), prv)
            out[f] += _spin(ID4 - sg * GAMMA[mu], fwd) + _spin(ID4 + sg * GAMMA[mu], bwd)
    return np.moveaxis(-0.5 * out, 0, -8)


def wilson(U, psi, M5, bc, adjoint=False):
    """D_W psi = (4 - M5) psi + Dhop psi (or its adjoint)."""
    return (4.0 - M5) * psi + hop(U, psi, bc, adjoint)


def chiral(psi, sign):
    """P_+ psi (sign=+1) or P_- psi (sign=-1)."""
    return _spin(P_PLUS if sign > 0 else P_MINUS, psi)


def gamma5(psi):
    return _spin(GAMMA5, psi)


def vdot(a, b):
    """<a, b> = sum conj(a) b."""
    return np.vdot(a.ravel(), b.ravel())


def norm2(a):
    return float(np.vdot(a.ravel(), a.ravel()).real)
