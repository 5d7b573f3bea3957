"""Pins of the statistics oracle against closed forms and independent
counts: central-difference dissipation of a shear wave and of linear fields
(shear, strain, rigid rotation), Parseval for the spectrum, the decay of a
lattice shear wave (-dE/dt = eps), lattice-point counts of the distance bins,
masking by the rigid-body motion, and particle energies."""
import math

import numpy as np

from oracle import stats
from oracle.sim import Config, Sim


def _linear_field(shape, A):
    """u_i = sum_j A[i, j] x_j (not periodic: only interior nodes are exact)."""
    xyz = stats.node_coords(shape)
    return np.einsum("ij,j...->i...", A, xyz)


def test_shear_wave_dissipation_closed_form():
    """u_x = a sin(k y): the central difference gives a cos(k y) sin(k), so
    eps(x) = 2 nu (2 (a cos(ky) sin(k) / 2)^2) and <eps> = nu a^2 sin(k)^2 / 2."""
    shape = (6, 40, 5)
    nu, a, m = 0.02, 0.013, 3
    k = 2 * np.pi * m / shape[1]
    y = np.arange(shape[1])
    u = np.zeros((3, shape[2], shape[1], shape[0]))
    u[0] = a * np.sin(k * y)[None, :, None]
    eps = stats.dissipation_field(u, nu)
    want = nu * (a * np.cos(k * y) * np.sin(k)) ** 2
    assert np.allclose(eps, want[None, :, None], rtol=1e-12, atol=1e-12 * want.max())
    s = stats.statistics(u, np.ones(u.shape[1:]), nu, shape)
    assert math.isclose(s["eps_raw"], nu * a * a * np.sin(k) ** 2 / 2, rel_tol=1e-12)
    assert math.isclose(s["ke_raw"], a * a / 4, rel_tol=1e-12)


def test_linear_shear_pure_strain_and_rotation():
    """Central differences are exact on linear fields: simple shear u_x =
    g y gives eps = nu g^2; pure strain (a x, -a y, 0) gives 4 nu a^2; a rigid
    rotation (antisymmetric gradient) dissipates nothing."""
    shape = (9, 8, 7)
    nu = 0.01
    inner = (slice(1, -1),) * 3
    g = 0.003
    A = np.zeros((3, 3))
    A[0, 1] = g
    eps = stats.dissipation_field(_linear_field(shape, A), nu)[inner]
    assert np.allclose(eps, nu * g * g, rtol=1e-12, atol=0)
    A = np.diag([0.002, -0.002, 0.0])
    eps = stats.dissipation_field(_linear_field(shape, A), nu)[inner]
    assert np.allclose(eps, 4 * nu * 0.002 ** 2, rtol=1e-12, atol=0)
    Om = np.array([0.001, -0.002, 0.0015])
    A = np.array([[0, -Om[2], Om[1]], [Om[2], 0, -Om[0]], [-Om[1], Om[0], 0]])
    eps = stats.dissipation_field(_linear_field(shape, A), nu)[inner]
    assert np.abs(eps).max() < 1e-20
    # a general gradient: eps = nu |A + A^T|^2 / 2
    A = np.random.default_rng(1).normal(size=(3, 3)) * 1e-3
    eps = stats.dissipation_field(_linear_field(shape, A), nu)[inner]
    assert np.allclose(eps, 0.5 * nu * ((A + A.T) ** 2).sum(), rtol=1e-12, atol=0)


def test_spectrum_parseval_and_shell_of_single_mode():
    rng = np.random.default_rng(4)
    u = rng.normal(size=(3, 10, 12, 14))
    k, E = stats.energy_spectrum(u)
    assert math.isclose(E.sum(), 0.5 * (u * u).sum(0).mean(), rel_tol=1e-12)
    # one Fourier mode (kx, ky, kz) = (3, 4, 0): all energy in shell 5
    shape = (16, 16, 8)
    xyz = stats.node_coords(shape)
    v = np.zeros((3,) + xyz.shape[1:])
    v[2] = 0.01 * np.cos(2 * np.pi * (3 * xyz[0] / 16 + 4 * xyz[1] / 16))
    k, E = stats.energy_spectrum(v)
    assert np.argmax(E) == 5 and math.isclose(E[5], 0.25 * 0.01 ** 2, rel_tol=1e-12)
    assert E.sum() - E[5] < 1e-20
    D = stats.dissipation_spectrum(k, E, 0.1)
    assert math.isclose(D[5], 2 * 0.1 * 25 * E[5], rel_tol=1e-14)


def test_lattice_shear_wave_energy_decay_matches_dissipation():
    """Unforced periodic shear wave on the FP64 lattice Boltzmann oracle: the
    energy decays at the rate the dissipation statistic reports, up to the
    O(k^2) difference between the central difference and the exact
    derivative."""
    shape = (4, 64, 4)
    tau = 0.8
    nu = (tau - 0.5) / 3
    sim = Sim(Config(shape=shape, tau=tau))
    y = np.arange(shape[1])
    k = 2 * np.pi / shape[1]
    u = np.zeros((3, shape[2], shape[1], shape[0]))
    u[0] = 0.01 * np.sin(k * y)[None, :, None]
    sim.set_fields(u)
    sim.step(20)
    E, eps = [], []
    for _ in range(3):
        uu, rr = sim.fields()
        s = stats.statistics(uu, rr, nu, shape)
        E.append(s["ke_raw"])
        eps.append(s["eps_raw"])
        sim.step(1)
    dEdt = (E[2] - E[0]) / 2
    assert abs(-dEdt - eps[1]) < 0.01 * eps[1]


def _count_in_sphere(X, R, shape):
    """Lattice points with periodic distance < R by slices: for each (y, z)
    row, the x range is an interval whose ends come from a square root."""
    nx, ny, nz = shape
    n = 0
    for z in range(nz):
        dz = min((z - X[2]) % nz, (X[2] - z) % nz)
        for y in range(ny):
            dy = min((y - X[1]) % ny, (X[1] - y) % ny)
            rem = R * R - dy * dy - dz * dz
            if rem <= 0:
                continue
            h = math.sqrt(rem)
            lo, hi = math.floor(X[0] - h) + 1, math.ceil(X[0] + h) - 1
            n += max(0, hi - lo + 1)
    return n


def test_distance_bins_count_lattice_points_in_shells():
    shape = (40, 36, 38)
    X = np.array([[17.3, 18.6, 19.1]])
    r = np.array([6.2])
    nb = 12
    owner, b = stats.classify(shape, X, r, nbins=nb)
    inside = _count_in_sphere(X[0], r[0], shape)
    assert (owner == 0).sum() == inside
    for j in range(nb):
        shell = _count_in_sphere(X[0], r[0] + (j + 1) * stats.BIN_WIDTH, shape) - \
            _count_in_sphere(X[0], r[0] + j * stats.BIN_WIDTH, shape)
        assert (b == j).sum() == shell, j
    # every node is either inside, binned or beyond the last bin
    far = _count_in_sphere(X[0], r[0] + nb * stats.BIN_WIDTH, shape)
    assert (b < 0).sum() == owner.size - far + inside


def test_nearest_surface_counts_each_node_once():
    """Two spheres: a node takes the bin of the nearer surface."""
    shape = (48, 24, 24)
    X = np.array([[12.2, 12.1, 11.7], [33.9, 12.4, 12.2]])
    r = np.array([5.0, 7.5])
    owner, b = stats.classify(shape, X, r, nbins=80)
    xyz = stats.node_coords(shape)
    for node in [(22, 12, 12), (24, 12, 12), (25, 12, 12), (23, 3, 20)]:
        x, y, z = node
        d = [math.dist((x, y, z), X[p]) - r[p] for p in range(2)]
        assert b[z, y, x] == math.floor(min(d) / stats.BIN_WIDTH)
    assert xyz.shape == (3, 24, 24, 48)


def test_masking_rigid_motion_and_pipe():
    shape = (30, 28, 26)
    X = np.array([[10.5, 12.0, 13.3]])
    U = np.array([[0.01, -0.02, 0.005]])
    Om = np.array([[0.001, 0.0, -0.002]])
    u = np.random.default_rng(2).normal(size=(3, 26, 28, 30)) * 0.01
    owner, _ = stats.classify(shape, X, np.array([4.0]))
    um = stats.masked_velocity(u, owner, X, U, Om, shape)
    sel = owner == 0
    assert sel.sum() > 200
    x = (10, 12, 13)
    d = np.array(x) - X[0]
    assert np.allclose(um[:, 13, 12, 10], U[0] + np.cross(Om[0], d), rtol=0, atol=1e-16)
    assert np.array_equal(um[:, ~sel], u[:, ~sel])
    # rigid motion inside leaves the gradient zero deep inside: no dissipation there
    eps = stats.dissipation_field(um, 0.01)
    assert eps[13, 12, 10] < 1e-20
    # pipe: solid outside R, radial bins of the wall distance
    owner, b = stats.classify(shape, np.zeros((0, 3)), np.zeros(0), pipe=(10.0, 14.5, 13.5), nbins=80)
    assert (owner == -2).sum() == owner.size - 26 * _count_disc(10.0, 14.5, 13.5, shape)
    um = stats.masked_velocity(u, owner, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)), shape)
    assert np.abs(um[:, owner == -2]).max() == 0.0
    assert b[0, 13, 14] == math.floor((10.0 - math.hypot(0.5, 0.5)) / stats.BIN_WIDTH)


def _count_disc(R, cx, cy, shape):
    nx, ny, _ = shape
    return sum(1 for y in range(ny) for x in range(nx) if (x - cx) ** 2 + (y - cy) ** 2 < R * R)


def test_uniform_flow_sums_and_particle_energies():
    shape = (12, 10, 14)
    Uf = np.array([0.02, -0.01, 0.03])
    u = np.broadcast_to(Uf[:, None, None, None], (3, 14, 10, 12)).copy()
    rho = np.full((14, 10, 12), 1.01)
    X = np.array([[5.0, 5.0, 6.0]])
    Up = np.array([[0.003, 0.0, 0.0]])
    Om = np.array([[0.0, 0.0, 0.002]])
    s = stats.statistics(u, rho, 0.01, shape, X, Up, Om, np.array([3.0]), np.array([4.0]))
    nf = s["n_fluid"]
    assert nf == u[0].size - _count_in_sphere(X[0], 3.0, shape)
    assert math.isclose(s["mass"], 1.01 * nf, rel_tol=1e-13)
    assert np.allclose(s["momentum"], 1.01 * nf * Uf, rtol=1e-13)
    assert math.isclose(s["ke_fluid"], 0.5 * (Uf * Uf).sum(), rel_tol=1e-13)
    assert math.isclose(s["ke_raw"], 0.5 * (Uf * Uf).sum(), rel_tol=1e-13)
    assert s["eps_raw"] < 1e-30
    assert math.isclose(s["bulk_u"], 0.03, rel_tol=1e-13)
    assert math.isclose(s["umax"], np.linalg.norm(Uf), rel_tol=1e-13)
    m = 4.0 * 4.0 / 3.0 * math.pi * 27.0
    assert math.isclose(s["particle_ke"], 0.5 * m * 0.003 ** 2, rel_tol=1e-13)
    assert math.isclose(s["particle_ke_rot"], 0.5 * 0.4 * m * 9.0 * 0.002 ** 2, rel_tol=1e-13)
    h = s["hist"]
    assert np.allclose(h[1], h[0] * 0.5 * (Uf * Uf).sum(), rtol=1e-12)
    assert np.allclose(h[3], h[0] * 0.03, rtol=1e-12)
