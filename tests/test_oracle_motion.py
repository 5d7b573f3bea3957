"""Pins of the oracle's refill, release, rotational dynamics and torque
arithmetic against facts fixed outside it:

* refill (Sec. 3.1): polynomial exactness of the three- and two-point
  extrapolations along the lattice direction nearest the outward normal,
  the wall-velocity substitution, the neighbour-average fallback;
* release (Sec. 3.1): the solid-fraction-weighted volume average of the
  fluid velocity, Omega = 0, the interior reset to the rigid motion;
* rotation: Omega' - Omega = T / I with I the moment of inertia of a solid
  ball, obtained here by numerical quadrature;
* torques: the exact lattice angular-momentum budget of a fixed sphere for
  bounce-back links (their lever arms and signs) and for the immersed
  boundary (marker torques plus the Kempe term), and the Kempe angular
  integral of a rigid rotation against the ball's inertia tensor;
* drag (Sec. 3.1, the periodic sphere array): the oracle's bounce-back
  drag of a simple cubic array in creeping flow against the
  Hasimoto / Sangani-Acrivos series."""
import itertools
import math

import numpy as np
import pytest

from oracle import collide as col
from oracle import geometry as geo
from oracle import ibm, refill
from oracle.lattice import C, CF
from oracle.particles import Particles, advance
from oracle.sim import RELEASE, SET_RIGID, Config, Sim

DIRS = [np.array(c) for c in itertools.product((-1, 0, 1), repeat=3) if 1 <= sum(abs(v) for v in c) <= 2]


def _expected_direction(d):
    """Brute force over the 18 moving directions: the largest c . d, ties to
    the lexicographically largest c; returns the direction and whether the
    maximum was unique."""
    vals = sorted(((float(np.dot(c, d)), tuple(int(v) for v in c)) for c in DIRS), reverse=True)
    return np.array(vals[0][1]), vals[0][0] > vals[1][0]


def _one_particle(X, U, Om=(0.0, 0.0, 0.0)):
    return Particles(np.array([X], float), np.array([U], float), np.array([Om], float), np.array([4.0]),
                     np.array([1.0]))


def _field(shape, fn):
    """Populations (19, z, y, x) from fn(x, y, z) -> (19,)."""
    nx, ny, nz = shape
    f = np.empty((19, nz, ny, nx))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                f[:, z, y, x] = fn(np.array([x, y, z], float))
    return f


def test_refill_three_point_exact_for_quadratic_equilibrium_field():
    """f = f_eq(1, u(x)) with u affine in x is quadratic in x, so the
    three-point extrapolation 3 f1 - 3 f2 + f3 reproduces f at the node
    exactly; with u_w = u(node) the refill returns that value, and with any
    other u_w it differs from it by f_eq(1, u_w) - f_eq(1, u(node))."""
    shape = (16, 16, 16)
    G = np.array([[0.004, -0.002, 0.003], [0.001, 0.005, -0.004], [-0.003, 0.002, 0.001]])
    u0 = np.array([0.02, -0.01, 0.015])
    x0 = np.array([8, 8, 8])
    uf = lambda x: u0 + G @ (x - x0)
    ft = _field(shape, lambda x: col.equilibrium(1.0, uf(x)))
    valid = np.ones((16, 16, 16), bool)
    valid[8, 8, 8] = False
    for d in ([2.8, 0.3, -0.1], [-0.2, -2.6, 1.9], [0.1, 0.4, -3.0]):
        X = x0 - np.array(d)
        ck, unique = _expected_direction(np.array(d))
        assert unique
        assert np.array_equal(C[refill.extrapolation_direction(np.array(d))], ck)
        # u_w equal to the field velocity at the node: the field value itself
        P = _one_particle(X, uf(x0))
        got = refill.refill_node(ft, valid, tuple(x0), 0, P, shape)
        assert np.abs(got - col.equilibrium(1.0, uf(x0))).max() < 1e-15
        # another wall velocity: only the equilibrium part changes
        uw = uf(x0) + np.array([0.01, -0.02, 0.005])
        P = _one_particle(X, uw)
        got = refill.refill_node(ft, valid, tuple(x0), 0, P, shape)
        want = col.equilibrium(1.0, uw)
        assert np.abs(got - want).max() < 1e-15
        assert abs(got.sum() - 1.0) < 1e-15
        assert np.abs(CF.T @ got - uw).max() < 1e-15


def test_refill_two_point_exact_along_the_normal_only():
    """Only x + c_k and x + 2 c_k valid (x + 3 c_k holds NaN): the two-point
    rule 2 f1 - f2 is exact for a field linear in x, equilibrium or not.
    Any other direction, the three-point rule or the neighbour average would
    read NaN or miss the exact value."""
    shape = (16, 16, 16)
    rng = np.random.default_rng(4)
    a = rng.normal(scale=1e-3, size=19)
    B = rng.normal(scale=2e-4, size=(19, 3))
    x0 = np.array([8, 8, 8])
    base = col.equilibrium(1.0, np.array([0.01, 0.02, -0.01]))
    lin = lambda x: base + a + B @ (x - x0)
    for d in ([1.7, -2.2, 0.4], [0.3, 0.2, 2.9], [-2.5, 0.1, -2.0]):
        ck, unique = _expected_direction(np.array(d))
        assert unique
        ft = np.full((19, 16, 16, 16), np.nan)
        valid = np.zeros((16, 16, 16), bool)
        for s in (1, 2):
            x = x0 + s * ck
            ft[:, x[2], x[1], x[0]] = lin(x.astype(float))
            valid[x[2], x[1], x[0]] = True
        f_node = lin(x0.astype(float))
        rho = f_node.sum()
        u_node = CF.T @ f_node / rho
        P = _one_particle(x0 - np.array(d), u_node)
        got = refill.refill_node(ft, valid, tuple(x0), 0, P, shape)
        assert np.abs(got - f_node).max() < 1e-15


def test_refill_neighbour_average_and_last_fallback():
    """No extrapolation along the normal (x + 2 c_k invalid): the average
    density and velocity of the valid nearest neighbours, at equilibrium,
    with the velocity replaced by u_w; no valid neighbour: f_eq(1, u_w)."""
    shape = (12, 12, 12)
    rho0, ua = 1.013, np.array([0.02, -0.015, 0.01])
    feq0 = col.equilibrium(rho0, ua)
    x0 = np.array([6, 6, 6])
    d = np.array([0.2, 2.7, 0.4])
    ck, _ = _expected_direction(d)
    ft = np.full((19, 12, 12, 12), np.nan)
    valid = np.zeros((12, 12, 12), bool)
    for c in DIRS[::3]:
        x = x0 + c
        if np.array_equal(c, ck):
            continue
        ft[:, x[2], x[1], x[0]] = feq0
        valid[x[2], x[1], x[0]] = True
    x1 = x0 + ck
    ft[:, x1[2], x1[1], x1[0]] = feq0
    valid[x1[2], x1[1], x1[0]] = True
    uw = np.array([-0.01, 0.03, 0.0])
    got = refill.refill_node(ft, valid, tuple(x0), 0, _one_particle(x0 - d, uw), shape)
    assert np.abs(got - col.equilibrium(rho0, uw)).max() < 1e-15
    valid[:] = False
    got = refill.refill_node(ft, valid, tuple(x0), 0, _one_particle(x0 - d, uw), shape)
    assert np.abs(got - col.equilibrium(1.0, uw)).max() < 1e-15


def _release(shape, u, X, r, bc="ibb"):
    sim = Sim(Config(shape=shape, tau=0.6, bc=bc))
    sim.set_fields(u)
    sim.set_particles([X], r=[r], Om=[[0.01, -0.02, 0.03]], mode=RELEASE)
    return sim


def _dist(shape, X):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = [geo.min_image(x - X[0], nx), geo.min_image(y - X[1], ny), geo.min_image(z - X[2], nz)]
    return np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2), np.stack(d)


@pytest.mark.parametrize("bc", ["ibb", "ibm"])
def test_release_velocity_is_the_weighted_volume_average(bc):
    """Release (Sec. 3.1): U0 averages the fluid velocity over the particle
    with the cell solid fraction as weight, Omega0 = 0.
    (1) a uniform flow gives U exactly; (2) the velocity beyond the reach of
    any partly covered cell (|x - X| >= r + sqrt(3)/2) does not enter;
    (3) with u = U_a + b on the nodes whose whole cell is inside (weight 1),
    U0 - U_a = b N_deep / sum(weights) and the weights add up to the ball's
    volume, so an unweighted mean over the covered cells (27% off at r = 8)
    fails."""
    shape = (28, 28, 28)
    X, r = np.array([13.6, 14.2, 13.9]), 8.0
    dist, _ = _dist(shape, X)
    Ua = np.array([0.013, -0.021, 0.008])
    u = np.broadcast_to(Ua[:, None, None, None], (3, 28, 28, 28)).copy()
    sim = _release(shape, u, X, r, bc)
    assert np.abs(sim.state.P.U[0] - Ua).max() < 1e-15
    assert np.all(sim.state.P.Om == 0.0)
    far = dist >= r + 0.8661
    u[:, far] = np.array([5.0, -3.0, 7.0])[:, None]
    sim = _release(shape, u, X, r, bc)
    assert np.abs(sim.state.P.U[0] - Ua).max() < 1e-14
    u[:, far] = Ua[:, None]
    deep = dist < r - 0.8661  # all 8 corners of the cell inside
    b = np.array([0.01, 0.02, -0.03])
    u[:, deep] += b[:, None]
    sim = _release(shape, u, X, r, bc)
    vol = 4.0 / 3.0 * math.pi * r ** 3
    want = b * deep.sum() / vol
    got = sim.state.P.U[0] - Ua
    # the weights add up to the volume within the fraction's O(dx^2) error
    assert np.abs(got - want).max() < 1e-2 * np.abs(want).max()
    covered = dist < r + 0.8661
    unweighted = b * deep.sum() / covered.sum()
    assert np.abs(unweighted - want).max() > 0.2 * np.abs(want).max()
    # (4) cells whose node lies outside the sphere but whose cell is partly
    # covered carry a positive weight below one: a node-inside indicator
    # would give them none
    u[:, deep] -= b[:, None]
    shell = (dist >= r) & covered
    u[:, shell] += b[:, None]
    sim = _release(shape, u, X, r, bc)
    frac = (sim.state.P.U[0] - Ua) / b
    assert np.abs(frac - frac[0]).max() < 1e-12
    assert 0.01 < frac[0] < shell.sum() / (4.0 / 3.0 * math.pi * r ** 3)


def test_release_resets_interior_to_rigid_motion():
    """SET_RIGID (and RELEASE with its averaged U): the populations at
    interior nodes become the equilibrium of the local density and the
    rigid-body velocity U + Omega x (x - X)."""
    shape = (24, 24, 24)
    X, r = np.array([11.3, 12.6, 12.1]), 6.0
    rho = 1.0 + 0.01 * np.random.default_rng(2).standard_normal((24, 24, 24))
    sim = Sim(Config(shape=shape, tau=0.6, bc="ibm"))
    sim.set_fields(np.zeros((3, 24, 24, 24)), rho)
    U, W = np.array([0.01, 0.0, -0.02]), np.array([0.002, -0.001, 0.003])
    sim.set_particles([X], U=[U], Om=[W], r=[r], mode=SET_RIGID)
    dist, d = _dist(shape, X)
    inside = dist < r
    ft = sim.state.ft
    urig = U[:, None] + np.cross(W, d[:, inside].T).T
    want = col.equilibrium(rho[inside], urig)
    assert np.abs(ft[:, inside] - want).max() < 1e-15
    assert np.abs(ft[:, ~inside] - col.equilibrium(rho[~inside], np.zeros((3, (~inside).sum())))).max() < 1e-15


def _ball_inertia_quadrature(r, rho, n=161):
    """I_zz = rho * integral over the ball of (x^2 + y^2), midpoint rule with
    each cell weighted by its covered fraction on a 4^3 subgrid."""
    h = 2.0 * r / n
    c = -r + h * (np.arange(n) + 0.5)
    sub = (np.arange(4) + 0.5) / 4.0 - 0.5
    tot = 0.0
    for sz in sub:
        for sy in sub:
            z = (c + sz * h)[:, None, None]
            y = (c + sy * h)[None, :, None]
            x = (c[None, None, :] + sub[:, None, None, None] * h)
            inside = (x * x + y * y + z * z) < r * r
            tot += ((x * x + y * y) * inside).sum()
    return rho * tot * h ** 3 / 64.0


def test_rotational_update_uses_the_solid_ball_inertia():
    """Omega' = Omega + T / I: an isolated torque on a free sphere changes
    Omega by T / I with I the moment of inertia of a solid ball of density
    rho_p (numerical quadrature here, 0.4 m r^2 in closed form), leaves U and
    X unchanged by rotation."""
    r, rho = 6.5, 3.0
    I = _ball_inertia_quadrature(r, rho)
    m = rho * 4.0 / 3.0 * math.pi * r ** 3
    assert abs(I / (0.4 * m * r * r) - 1.0) < 2e-3
    P = Particles(np.array([[10.0, 11.0, 12.0]]), np.array([[0.01, 0.0, 0.0]]), np.array([[0.0, 0.002, 0.0]]),
                  np.array([r]), np.array([rho]))
    T = np.array([[3.0, -1.5, 2.0]])
    P1 = advance(P, np.zeros((1, 3)), T, (64, 64, 64))
    assert np.abs((P1.Om - P.Om) * I / T - 1.0).max() < 2e-3
    assert np.array_equal(P1.U, P.U)
    assert np.abs(P1.X - (P.X + P.U)).max() < 1e-15


def _windowed_field(shape, X, radius, seed, amp=0.03):
    """Random velocity inside a smooth window of the given radius around X,
    rest (u = 0, rho = 1) beyond it."""
    rng = np.random.default_rng(seed)
    dist, _ = _dist(shape, X)
    win = np.where(dist < radius, np.cos(0.5 * np.pi * dist / radius) ** 2, 0.0)
    u = amp * rng.standard_normal((3,) + dist.shape) * win[None]
    rho = 1.0 + 0.005 * rng.standard_normal(dist.shape) * win
    return u, rho


def _angular_momentum(ft, X, shape, mask=None):
    """sum over nodes of (x - X) x j(x), j = sum c f (minimum-image arms)."""
    _, d = _dist(shape, X)
    j = col.momentum(ft)
    L = np.cross(d.reshape(3, -1).T, j.reshape(3, -1).T)
    if mask is not None:
        L = L[mask.ravel()]
    return L.sum(0), j.reshape(3, -1)[:, mask.ravel() if mask is not None else slice(None)].sum(1)


@pytest.mark.parametrize("max_order", [1, 2])
def test_ibb_fixed_sphere_angular_momentum_budget(max_order):
    """Streaming conserves sum x x c f (c x c = 0) and the collision conserves
    j at every node, so with a fixed sphere and the fluid at rest near the
    periodic faces the fluid's angular momentum about X changes each step by
    minus the link torques, to round-off. For a fixed wall every link force
    is parallel to its direction, so this holds for the wall-point lever arm
    x_w - X; a sign or arm error does not."""
    shape = (28, 28, 28)
    X, r = np.array([13.7, 14.2, 13.4]), 4.6
    u, rho = _windowed_field(shape, X, 7.5, seed=5)
    sim = Sim(Config(shape=shape, tau=0.6, bc="ibb", ibb_max_order=max_order))
    sim.set_fields(u, rho)
    sim.set_particles([X], r=[r], motion="fixed")
    fluid = sim.fluid_mask()
    L0, _ = _angular_momentum(np.where(fluid[None], sim.state.ft, 0.0), X, shape, fluid)
    Tsum = 0.0
    for _ in range(4):
        sim.step(1)
        _, T, _ = sim.forces()
        Tsum = Tsum + T[0]
        L1, _ = _angular_momentum(np.where(fluid[None], sim.state.ft, 0.0), X, shape, fluid)
        # round-off: the moment transforms of ~2e4 nodes, mostly identical
        # rest nodes whose rounding errors add up coherently
        assert np.abs(L1 - L0 + Tsum).max() < 3e-10
    assert np.abs(Tsum).max() > 1e-4


@pytest.mark.parametrize("rd", [0.0, 0.4])
def test_ibm_fixed_sphere_angular_momentum_and_force_budget(rd):
    """With the immersed boundary the whole lattice is fluid. The spread force
    changes the lattice momentum and angular momentum by exactly the sums of
    the marker forces and of their moments (Peskin's zeroth and first moment
    conditions), so F_h - dI_u = -dP and T_h - dI_L = -dL each step, with
    I_u, I_L the Kempe integrals (Sec. 3.1)."""
    shape = (28, 28, 28)
    X, r = np.array([13.7, 14.2, 13.4]), 4.6
    u, rho = _windowed_field(shape, X, 7.0, seed=6)
    sim = Sim(Config(shape=shape, tau=0.6, bc="ibm", ibm_retraction=rd))
    sim.set_fields(u, rho)
    sim.set_particles([X], r=[r], motion="fixed")
    L0, P0 = _angular_momentum(sim.state.ft, X, shape)
    for _ in range(3):
        Iu0, IL0 = sim.state.Iu.copy(), sim.state.IL.copy()
        sim.step(1)
        F, T, _ = sim.forces()
        L1, P1 = _angular_momentum(sim.state.ft, X, shape)
        dIu, dIL = sim.state.Iu[0] - Iu0[0], sim.state.IL[0] - IL0[0]
        assert np.abs((P1 - P0) + (F[0] - dIu)).max() < 3e-11
        assert np.abs((L1 - L0) + (T[0] - dIL)).max() < 3e-10
        assert np.abs(T[0] - dIL).max() > 1e-5
        L0, P0 = L1, P1


def test_kempe_angular_integral_of_rigid_rotation():
    """I_L = sum alpha (x - X) x u for u = Omega x (x - X) approximates
    integral over the ball of (|d|^2 Omega - d (d . Omega)) = (8 pi / 15)
    r^5 Omega; the relative error (mean over random centre offsets) falls
    with the radius at about second order in the spacing."""
    rng = np.random.default_rng(8)
    W = np.array([0.003, -0.002, 0.005])
    errs = []
    for r in (4.0, 8.0, 16.0):
        e = []
        for _ in range(3):
            shape = (48, 48, 48)
            X = 24.0 + rng.uniform(0, 1, 3)
            _, d = _dist(shape, X)
            u = np.cross(W, d.reshape(3, -1).T).T.reshape(d.shape)
            _, IL = ibm.inner_integrals(u, X[None], np.array([r]), shape)
            want = 8.0 * math.pi / 15.0 * r ** 5 * W
            e.append(np.abs(IL[0] - want).max() / np.abs(want).max())
        errs.append(np.mean(e))
    assert errs[-1] < 5e-3
    assert errs[1] < 0.5 * errs[0] and errs[2] < 0.5 * errs[1]


def _k_theory(phi):
    chi = phi ** (1.0 / 3.0)
    return 1.0 / (1.0 - 1.7601 * chi + chi ** 3 - 1.5593 * chi ** 6 + 3.9799 * chi ** 8 - 3.0734 * chi ** 10)


@pytest.mark.slow
def test_oracle_sphere_array_stokes_drag():
    """The oracle's quadratic bounce-back drag of a simple cubic array of fixed
    spheres in creeping flow (24^3 box, r = 3.375: the volume fraction of the
    32^3 / r = 4.5 configuration) against the Hasimoto / Sangani-Acrivos
    series K(phi): K = F / (6 pi mu a U_s) with U_s the superficial
    velocity, after the flow has settled (tau = 1 for a short spin-up)."""
    n, r, tau, gx = 24, 3.375, 1.0, 1e-7
    nu = (tau - 0.5) / 3.0
    phi = 4.0 / 3.0 * math.pi * r ** 3 / n ** 3
    sim = Sim(Config(shape=(n, n, n), tau=tau, body_force=(gx, 0.0, 0.0), bc="ibb"))
    sim.set_particles([[12.0, 12.0, 12.0]], r=[r], motion="fixed")
    fluid = sim.fluid_mask()
    # Start from the uniform flow whose superficial velocity balances the
    # body force at the series drag: only the local flow around the sphere
    # has to develop (time scale L^2 / (4 pi^2 nu) ~ 90 steps), not the mean
    # flow (V / (6 pi nu r K) ~ 800 steps).
    Us = gx * fluid.sum() / (6.0 * math.pi * nu * r * _k_theory(phi))  # superficial
    U0 = Us * n ** 3 / fluid.sum()                                        # interstitial
    sim.set_fields(np.broadcast_to(np.array([U0, 0.0, 0.0])[:, None, None, None], (3, n, n, n)))

    def K():
        F, _, _ = sim.forces()
        Us = float(np.where(fluid, sim.state.u[0], 0.0).sum()) / n ** 3
        return F[0, 0] / (6.0 * math.pi * nu * r * Us)

    sim.step(500)
    K1 = K()
    sim.step(100)
    K2 = K()
    ratio = K2 / _k_theory(phi)
    print(f"oracle sphere array: K {K2:.4f}, K_theory {_k_theory(phi):.4f}, ratio {ratio:.4f}, "
          f"change {abs(K2 - K1) / K2:.1e}")
    assert abs(K2 - K1) < 2e-3 * K2
    assert 0.95 < ratio < 1.08
