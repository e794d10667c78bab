"""Seeded synthetic inputs: SU(3) gauge fields and Gaussian fermion fields.

This module holds none of the solver's arithmetic. It is the only code the
GPU path and the CPU oracle share: both receive the same arrays from here.

Recipe (the paper's ensembles are not available; these stand in for them):

* links U = exp(i eps H) with H = sum_a h_a lambda_a / 2, h_a ~ N(0, 1)
  i.i.d. and lambda_a the Gell-Mann matrices; the exponential is taken
  through the eigen-decomposition of the Hermitian H, so U is unitary
  with unit determinant to rounding;
* fermion sources: real and imaginary parts i.i.d. N(0, 1/2) (the
  normalisation the paper uses for the heatbath draw eta);
* numpy PCG64 streams (``numpy.random.default_rng(seed)``).

Host arrays are complex128 in the canonical layouts
``[4, T, Z, Y, X, 3, 3]`` (gauge) and ``[..., Ls, T, Z, Y, X, 4, 3]``
(fermion). Large fields can be drawn directly on a device with
``fermion_torch`` (torch's seeded generator, same distribution).
"""
import numpy as np

_GM = np.zeros((8, 3, 3), dtype=np.complex128)
_GM[0][0, 1] = _GM[0][1, 0] = 1
_GM[1][0, 1], _GM[1][1, 0] = -1j, 1j
_GM[2][0, 0], _GM[2][1, 1] = 1, -1
_GM[3][0, 2] = _GM[3][2, 0] = 1
_GM[4][0, 2], _GM[4][2, 0] = -1j, 1j
_GM[5][1, 2] = _GM[5][2, 1] = 1
_GM[6][1, 2], _GM[6][2, 1] = -1j, 1j
_GM[7][0, 0] = _GM[7][1, 1] = 1 / np.sqrt(3)
_GM[7][2, 2] = -2 / np.sqrt(3)
GELL_MANN = _GM


def _su3_exp(h, eps):
    """exp(i eps sum_a h_a lambda_a / 2) for h[..., 8]."""
    H = np.einsum("...a,aij->...ij", h, GELL_MANN) / 2.0
    w, V = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", V, ph, V.conj())


def gauge_field(dims, eps, seed):
    """Links exp(i eps H) on a lattice dims = (Lx, Ly, Lz, Lt)."""
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    out = np.empty((4, lt, lz, ly, lx, 3, 3), dtype=np.complex128)
    for mu in range(4):
        h = rng.standard_normal((lt, lz, ly, lx, 8))
        out[mu] = _su3_exp(h, eps)
    return out


def unit_gauge(dims):
    lx, ly, lz, lt = dims
    u = np.zeros((4, lt, lz, ly, lx, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def gauge_transform(dims, seed, eps=2.0):
    """Random site field g(x) in SU(3), [T, Z, Y, X, 3, 3]."""
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    return _su3_exp(rng.standard_normal((lt, lz, ly, lx, 8)), eps)


def fermion(dims, Ls, seed, nrhs=None, sigma2=0.5):
    """Gaussian complex field [nrhs?, Ls, T, Z, Y, X, 4, 3]."""
    lx, ly, lz, lt = dims
    shape = (Ls, lt, lz, ly, lx, 4, 3)
    if nrhs is not None:
        shape = (nrhs,) + shape
    rng = np.random.default_rng(seed)
    sd = np.sqrt(sigma2)
    return rng.normal(0.0, sd, shape) + 1j * rng.normal(0.0, sd, shape)


def fermion_torch(dims, Ls, seed, nrhs=1, device="cuda", sigma2=0.5):
    """Same distribution drawn on a device with torch's seeded generator
    (for fields too large to build on the host)."""
    import torch
    lx, ly, lz, lt = dims
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    shape = (nrhs, Ls, lt, lz, ly, lx, 4, 3, 2)
    x = torch.randn(shape, generator=g, device=device, dtype=torch.float64)
    x.mul_(float(np.sqrt(sigma2)))
    return torch.view_as_complex(x)
