"""Pins of the G-parity reading (x direction) of the oracle's hop.

The paper uses G-parity ensembles but gives no operator form; the reading
(flavour-doubled fields, conj(U) for flavour 1, twist Tw = [[0, 1], [-1, 0]]
across the x edge, links U(x + L) = conj(U(x))) is pinned by:
* the free-field spectrum: eigenvalues of D_W equal (4 - M5) - sum cos p +- i|sin p|
  with p_x = (2n + 1) pi / (2 L_x), n = 0 .. 2 L_x - 1 (the twist has
  eigenvalues +-i), p_y, p_z periodic and p_t antiperiodic;
* gamma_5 hermiticity and the adjoint with random links;
* gauge covariance under G-parity-compatible transforms (conj(g) on
  flavour 1, g(x + L) = conj(g(x)));
* equality with the ordinary Wilson hop on the x-doubled lattice
  [U, conj(U)] with an antiperiodic x edge (the form the library builds).
"""
import numpy as np

from oracle.lattice import hop, vdot, gamma5, dagger, shift, GAMMA
from oracle import reference
from paper_1706_05843_amd import synth

M5 = 1.8


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_free_spectrum():
    dims = (4, 2, 2, 2)
    lx, ly, lz, lt = dims
    bc = (2, 1, 1, -1)
    U = synth.unit_gauge(dims)
    shape = (2, 1, lt, lz, ly, lx, 4, 3)
    D = reference.dense_matrix(lambda x: (4.0 - M5) * x + hop(U, x, bc), shape)
    ev = np.linalg.eigvals(D)
    ref = []
    for nx in range(2 * lx):
        for ny in range(ly):
            for nz in range(lz):
                for nt in range(lt):
                    p = [(2 * nx + 1) * np.pi / (2 * lx), 2 * np.pi * ny / ly, 2 * np.pi * nz / lz,
                         (2 * nt + 1) * np.pi / lt]
                    a = 4.0 - M5 - sum(np.cos(q) for q in p)
                    b = np.sqrt(sum(np.sin(q) ** 2 for q in p))
                    ref += [a + 1j * b] * 6 + [a - 1j * b] * 6
    key = lambda z: (round(z.real, 8), round(z.imag, 8))
    assert len(ev) == len(ref)
    assert np.abs(np.array(sorted(ev, key=key)) - np.array(sorted(ref, key=key))).max() < 1e-10


def test_hermiticity_and_adjoint():
    dims = (4, 2, 2, 4)
    bc = (2, 1, 1, -1)
    U = synth.gauge_field(dims, 0.7, seed=5)
    shape = (2, 2, dims[3], dims[2], dims[1], dims[0], 4, 3)
    a, b = _rand(shape, 1), _rand(shape, 2)
    lhs = vdot(a, hop(U, b, bc))
    assert abs(lhs - vdot(gamma5(hop(U, gamma5(a), bc)), b)) < 1e-13 * abs(lhs)
    assert abs(lhs - vdot(hop(U, a, bc, adjoint=True), b)) < 1e-13 * abs(lhs)


def test_gauge_covariance():
    dims = (4, 2, 2, 2)
    bc = (2, 1, 1, -1)
    L = dims[0]
    U = synth.gauge_field(dims, 0.7, seed=7)
    g = synth.gauge_transform(dims, seed=8)
    Ug = np.empty_like(U)
    for mu in range(4):
        gn = shift(g, mu, +1)
        if mu == 0:  # g(x + L) = conj(g(x)) across the edge
            gn[..., L - 1, :, :] = np.conj(g[..., 0, :, :])
        Ug[mu] = g @ U[mu] @ dagger(gn)
    psi = _rand((2, 1, dims[3], dims[2], dims[1], dims[0], 4, 3), 9)
    G = lambda f: np.stack([np.einsum("...ab,...sb->...sa", g, f[0]),
                            np.einsum("...ab,...sb->...sa", np.conj(g), f[1])])
    a = hop(Ug, G(psi), bc)
    b = G(hop(U, psi, bc))
    assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()


def test_equals_doubled_lattice():
    dims = (4, 2, 2, 2)
    lx = dims[0]
    bc = (2, 1, 1, -1)
    U = synth.gauge_field(dims, 0.7, seed=11)
    psi = _rand((2, 1, dims[3], dims[2], dims[1], lx, 4, 3), 12)
    got = hop(U, psi, bc)
    U2 = np.concatenate([U, np.conj(U)], axis=-3)   # links of x' = x + f L
    psi2 = np.concatenate([psi[0], psi[1]], axis=-3)
    out2 = hop(U2, psi2, (-1.0, 1.0, 1.0, -1.0))
    ref = np.stack([out2[..., :lx, :, :], out2[..., lx:, :, :]])
    assert np.abs(got - ref).max() < 1e-14 * np.abs(ref).max()


def test_eofa_solve_with_gparity():
    """On a 2^4 x Ls=4 G-parity lattice the EOFA system matrix stays Hermitian
    and the paper's route (mirror mode) reproduces dense LU."""
    from oracle import eo
    from oracle.dwf import Action, System, H_system
    from oracle.lattice import norm2
    act = Action((2, 2, 2, 2), 4, M5, 1.5, 0.5, (2, 1, 1, -1))
    U = synth.gauge_field(act.dims, 0.4, seed=21)
    sysm = System(1.0, 0.04, 1.0, -1.0, +1)
    H = reference.dense_matrix(lambda x: H_system(act, U, sysm, x), act.field_shape)
    assert np.abs(H - H.conj().T).max() < 1e-13
    phi = _rand(act.field_shape, 22)
    x_dense = np.linalg.solve(H, phi.ravel()).reshape(phi.shape)
    out = eo.solve_mirror(act, U, sysm, phi, tol=1e-13)
    assert np.sqrt(norm2(out["psi"] - x_dense) / norm2(x_dense)) < 1e-10
