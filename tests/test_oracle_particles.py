"""Pins of the oracle's particle machinery against facts fixed outside it:
brute-force link enumeration and bisection for q, Lagrange exactness of the
Bouzidi interpolants, exact Galilean invariance of a co-moving sphere,
the momentum budget of a fixed sphere, Peskin's delta-function moment
conditions, conservation of spread force and torque, the marker cell volume
and forcing-layer half-width the paper states, Kempe volume fractions,
and the closed-form restitution of the soft-sphere contact."""
import itertools
import math

import numpy as np
import pytest

from oracle import collide as col
from oracle import geometry as geo
from oracle import ibb, ibm
from oracle.lattice import C, CF, OPP, W
from oracle.particles import Particles, advance, contact_forces
from oracle.sim import Config, Sim

DIRS = [c for c in itertools.product((-1, 0, 1), repeat=3) if 1 <= sum(abs(v) for v in c) <= 2]


def _brute_owner(shape, X, r):
    nx, ny, nz = shape
    owner = {}
    for x in range(nx):
        for y in range(ny):
            for z in range(nz):
                inside = []
                for p in range(len(r)):
                    best = None
                    # minimum over the 27 periodic images
                    for sx in (-nx, 0, nx):
                        for sy in (-ny, 0, ny):
                            for sz in (-nz, 0, nz):
                                dx = (x - X[p][0]) + sx
                                dy = (y - X[p][1]) + sy
                                dz = (z - X[p][2]) + sz
                                d2 = (dx * dx + dy * dy) + dz * dz
                                best = d2 if best is None else min(best, d2)
                    if best < r[p] * r[p]:
                        inside.append(p)
                owner[(x, y, z)] = min(inside) if inside else -1
    return owner


def _bisect_q(d, c, r):
    lo, hi = 0.0, 1.0
    g = lambda t: sum((d[k] + t * c[k]) ** 2 for k in range(3)) - r * r
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_links_match_brute_force_on_tiny_grid():
    shape = (12, 10, 11)
    # one sphere straddles the x and z faces, two overlap each other
    X = np.array([[0.37, 4.61, 10.52], [6.2, 5.1, 5.3], [8.9, 5.6, 6.1]])
    r = np.array([2.7, 2.6, 2.2])
    brute = _brute_owner(shape, X, r)
    owner = geo.owner_map(shape, X, r)
    for (x, y, z), p in brute.items():
        assert owner[z, y, x] == p
    links = geo.build_links(owner, X, r, shape, max_order=2)
    got = sorted((int(p), int(x), int(y), int(z), tuple(C[a])) for (x, y, z), a, p in
                 zip(links["xf"], links["a"], links["p"]))
    exp = []
    nx, ny, nz = shape
    for (x, y, z), p in brute.items():
        if p != -1:
            continue
        for c in DIRS:
            s = brute[((x + c[0]) % nx, (y + c[1]) % ny, (z + c[2]) % nz)]
            if s != -1:
                exp.append((s, x, y, z, c))
    assert got == sorted(exp)
    # q against bisection on the minimum-image offset
    L = np.array(shape, float)
    for (x, y, z), a, p, q in zip(links["xf"], links["a"], links["p"], links["q"]):
        d = np.array([x, y, z], float) - X[p]
        d -= L * np.round(d / L)
        assert abs(q - _bisect_q(d, C[a], r[p])) < 1e-12
        assert 0.0 <= q < 1.0


def test_solid_count_close_to_sphere_volume():
    shape = (24, 24, 24)
    rng = np.random.default_rng(0)
    for rad in (4.5, 8.0):
        X = np.array([[12.0, 12.0, 12.0]]) + rng.uniform(0, 1, (1, 3))
        owner = geo.owner_map(shape, X, np.array([rad]))
        n = (owner == 0).sum()
        assert abs(n / (4 / 3 * np.pi * rad ** 3) - 1) < 0.03


def _one_link_case(q, scheme, fa, fb, uw=(0.0, 0.0, 0.0)):
    """ft with prescribed values along one link in direction a=1 (+x) from
    x_f = (4, 2, 2): fa[s] = f~_a(x_f - s c), fb[s] = f~_abar(x_f - s c)."""
    shape = (8, 5, 5)
    a = 1
    ft = np.full((19, 5, 5, 8), np.nan)
    for s in range(3):
        ft[a, 2, 2, 4 - s] = fa[s]
    for s in range(2):
        ft[OPP[a], 2, 2, 4 - s] = fb[s]
    links = {"xf": np.array([[4, 2, 2]]), "a": np.array([a]), "p": np.array([0]), "q": np.array([q]),
             "scheme": np.array([scheme])}
    return ibb.bounce_values(ft, links, np.array([uw]), shape)[0]


@pytest.mark.parametrize("q", [0.05, 0.2, 0.37, 0.5, 0.61, 0.83, 0.999])
def test_bouzidi_is_lagrange_exact(q):
    # Quadratic data g(s) = 1.3 - 0.7 s + 0.21 s^2 along the link (s = 0 at x_f,
    # s = 1 at x_f - c). For q < 1/2 the bounced population is f~_a carried
    # from s = 1 - 2q; for q >= 1/2 it is the abar field at s = 0 given its
    # values at s = 1 - 2q (the landing point of f~_a(x_f)), 1 and 2.
    g = lambda s: 1.3 - 0.7 * s + 0.21 * s * s
    h = lambda s: 0.4 + 0.11 * s                     # linear data
    if q < 0.5:
        v = _one_link_case(q, geo.SCHEME_QUADRATIC, [g(0), g(1), g(2)], [0, 0])
        assert abs(v - g(1 - 2 * q)) < 1e-13
        v = _one_link_case(q, geo.SCHEME_LINEAR, [h(0), h(1), np.nan], [0, 0])
        assert abs(v - h(1 - 2 * q)) < 1e-13
    else:
        v = _one_link_case(q, geo.SCHEME_QUADRATIC, [g(1 - 2 * q), np.nan, np.nan], [g(1), g(2)])
        assert abs(v - g(0)) < 1e-12
        v = _one_link_case(q, geo.SCHEME_LINEAR, [h(1 - 2 * q), np.nan, np.nan], [h(1), np.nan])
        assert abs(v - h(0)) < 1e-13


def test_bouzidi_reduces_to_halfway_bounce_back_at_half():
    fa = [0.21, 0.33, 0.17]
    fb = [0.29, 0.14]
    uw = (0.01, -0.02, 0.005)
    delta = -6 * W[1] * (CF[1] @ np.array(uw))
    for s in (geo.SCHEME_QUADRATIC, geo.SCHEME_LINEAR, geo.SCHEME_HALFWAY):
        assert abs(_one_link_case(0.5, s, fa, fb, uw) - (fa[0] + delta)) < 1e-15


def test_comoving_sphere_keeps_uniform_equilibrium():
    # Galilean invariance: a sphere carried by a uniform flow at its own
    # velocity leaves f = f_eq(1, U) everywhere (bounce-back, refill), and
    # the link forces sum to zero.
    shape = (16, 14, 15)
    U = np.array([0.021, -0.013, 0.008])
    sim = Sim(Config(shape=shape, tau=0.7, bc="ibb"))
    sim.set_particles([[7.3, 6.9, 7.6]], U=[U], r=[3.4], motion="prescribed")
    sim.set_fields(np.broadcast_to(U[:, None, None, None], (3,) + sim.cfg.zyx))
    feq = col.equilibrium(1.0, U)
    st = sim.state
    uw, arm = ibb.wall_velocity(st.links, st.P.X, st.P.U, st.P.Om, shape)
    fb = ibb.bounce_values(st.ft, st.links, uw, shape)
    Fl, _ = ibb.link_forces(st.ft, fb, st.links, uw, arm, shape)
    assert np.abs(Fl.sum(0)).max() < 1e-16 * np.abs(Fl).sum()
    refilled = 0
    for _ in range(60):
        sim.step(1)
        refilled += sim.state.extra["uncovered"]
        fl = sim.fluid_mask()
        assert np.abs(sim.state.ft[:, fl] - feq[:, None]).max() < 1e-14
    assert refilled > 20


def test_fixed_sphere_momentum_budget():
    # Fluid momentum changes by N_f g minus the link forces, every step.
    shape = (14, 13, 12)
    g = np.array([2e-5, -1e-5, 5e-6])
    sim = Sim(Config(shape=shape, tau=0.65, body_force=tuple(g), bc="ibb"))
    sim.set_particles([[6.4, 6.7, 5.2]], r=[3.3], motion="fixed")
    from synth import random_velocity
    sim.set_fields(random_velocity(shape, 0.02, seed=8))
    fluid = sim.fluid_mask()
    Nf = fluid.sum()

    def P():
        return col.momentum(np.where(fluid[None], sim.state.ft, 0.0)).reshape(3, -1).sum(1)

    for _ in range(6):
        p0 = P()
        sim.step(1)
        F, _, _ = sim.forces()
        # round-off of the moment transform leaves ~3e-16 per node
        assert np.allclose(P() - p0 + F[0], Nf * g, rtol=0, atol=1e-11)


def test_peskin_delta_moment_conditions():
    # Peskin 2002: sum_j phi(s-j) = 1, sum_j (s-j) phi(s-j) = 0,
    # sum_j phi(s-j)^2 = 3/8 for every shift s; support [-2, 2].
    for s in np.random.default_rng(1).uniform(0, 1, 50):
        j = np.arange(-3, 5)
        ph = ibm.peskin_phi(s - j)
        assert abs(ph.sum() - 1) < 1e-14
        assert abs(((s - j) * ph).sum()) < 1e-14
        assert abs((ph ** 2).sum() - 3 / 8) < 1e-14
    assert ibm.peskin_phi(np.array([2.0, -2.0, 2.3]))[:].max() == 0.0
    assert ibm.peskin_phi(np.array([1.999]))[0] > 0


def test_ibm_interpolation_exact_for_linear_fields_and_spread_conserves():
    shape = (24, 24, 24)
    rng = np.random.default_rng(2)
    xl = rng.uniform(6, 18, (40, 3))
    z, y, x = np.meshgrid(*[np.arange(24)] * 3, indexing="ij")
    A = rng.normal(size=(3, 3))
    b = rng.normal(size=3)
    u = np.stack([b[k] + A[k, 0] * x + A[k, 1] * y + A[k, 2] * z for k in range(3)])
    U = ibm.interpolate(u, xl, shape)
    assert np.abs(U - (b + xl @ A.T)).max() < 1e-12
    F = rng.normal(size=(40, 3))
    dV = rng.uniform(0.9, 1.1, 40)
    f = ibm.spread(F, dV, xl, shape)
    assert np.allclose(f.reshape(3, -1).sum(1), (F * dV[:, None]).sum(0), atol=1e-12)
    pos = np.stack([x, y, z]).reshape(3, -1)
    torque = np.cross(pos.T, f.reshape(3, -1).T).sum(0)
    assert np.allclose(torque, np.cross(xl, F * dV[:, None]).sum(0), atol=1e-10)


@pytest.mark.parametrize("r", [4.5, 8.0, 12.0])
def test_marker_volume_matches_cell_volume(r):
    # Sec. 2.1: the Lagrangian cell volume is about the Eulerian one.
    for rd in (0.0, 0.4):
        n = ibm.sphere_marker_count(r - rd)
        assert abs(ibm.sphere_marker_volume(r - rd, n) - 1.0) < 0.02
        d = ibm.fibonacci_directions(n)
        assert np.allclose((d * d).sum(1), 1.0)
        assert np.abs(d.mean(0)).max() < 2.0 / n


def test_marker_counts_of_the_configurations():
    # N_L = round(pi (12 r_L^2 + 1) / 3) for the radii used here: r = 8 and
    # r = 4.5 with markers on the surface or retracted by 0.4.
    assert [ibm.sphere_marker_count(rl) for rl in (8.0, 7.6, 4.5, 4.1)] == [805, 727, 256, 212]


def test_forcing_layer_fraction_printed_in_paper():
    # Sec. 3.2.1 prints the share of the particle volume inside the forcing
    # layer: 0.704 (d = 12 cells) and 0.421 (d = 24). A shell as thick as
    # the delta function's support half-width reproduces both.
    s = np.linspace(0, 3, 30001)
    half_width = s[ibm.peskin_phi(s) > 0].max()
    assert abs(half_width - 2.0) < 1e-3
    for d, printed in ((12, 0.704), (24, 0.421)):
        rp = d / 2
        assert round(1 - ((rp - round(half_width)) / rp) ** 3, 3) == printed


def test_multi_direct_forcing_converges():
    shape = (24, 24, 24)
    X = np.array([[11.7, 12.2, 12.4]])
    xl, own, arm, dV = ibm.sphere_markers(X, np.array([5.0]), 0.0, shape)
    Ud = np.tile([0.01, -0.004, 0.002], (len(xl), 1))
    u0 = np.zeros((3, 24, 24, 24))
    rho = np.ones((24, 24, 24))
    errs = []
    for passes in range(1, 13):
        _, u, _ = ibm.multi_direct_forcing(u0, rho, xl, Ud, dV, passes, shape)
        errs.append(np.abs(ibm.interpolate(u, xl, shape) - Ud).max())
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 0.05 * errs[0]


def test_kempe_fraction_integrates_to_volume():
    shape = (48, 48, 48)
    rng = np.random.default_rng(3)
    errs = []
    for r in (4.0, 8.0, 16.0):
        X = 24.0 + rng.uniform(0, 1, 3)
        nodes = geo.box_nodes(X, r + 1.0, shape)
        a = ibm.solid_fraction(X, r, nodes, shape)
        assert a.min() >= 0 and a.max() <= 1
        errs.append(abs(a.sum() / (4 / 3 * np.pi * r ** 3) - 1))
    assert errs[-1] < 2e-3 and errs[-1] < errs[0]


def test_soft_sphere_head_on_restitution_closed_form():
    # Isolated linear spring-dashpot contact: exit/entry normal speed = e and
    # contact lasts T_c (exact for the continuous equations; the explicit
    # step converges to it as T_c grows in steps).
    e, tc = 0.8, 400.0
    shape = (200.0, 200.0, 200.0)
    P = Particles(np.array([[90.0, 100.0, 100.0], [110.05, 100.0, 100.0]]),
                  np.array([[0.01, 0, 0], [-0.01, 0, 0]]), np.zeros((2, 3)),
                  np.array([10.0, 10.0]), np.array([1.0, 1.0]))
    v_in = 0.02
    t_contact = 0
    for _ in range(4000):
        F = contact_forces(P, shape, e, tc)
        if np.abs(F).max() > 0:
            t_contact += 1
        P = advance(P, F, np.zeros((2, 3)), shape)
        if t_contact and not np.abs(contact_forces(P, shape, e, tc)).max() and P.U[0, 0] < 0:
            break
    v_out = P.U[1, 0] - P.U[0, 0]
    assert abs(v_out / v_in - e) < 0.01
    assert abs(t_contact / tc - 1) < 0.02


def test_link_q_matches_bisection():
    """q from the cancellation-free root agrees with bisection on
    |x_f + t c - X|^2 = r^2 to 1e-12 for random links of random spheres."""
    from oracle.lattice import C
    rng = np.random.default_rng(17)
    checked = 0
    for _ in range(40):
        X = rng.random(3) * 2.0 + 10.0
        r = 2.0 + 4.0 * rng.random()
        for a in range(1, 19):
            c = np.array(C[a], float)
            # fluid node just outside, whose neighbour along c is inside
            for _ in range(5):
                d = rng.normal(size=3)
                d = d / np.linalg.norm(d) * (r + 0.3 * rng.random())
                xf = np.round(X + d)
                dv = xf - X
                if np.dot(dv, dv) < r * r or np.dot(dv + c, dv + c) >= r * r:
                    continue
                q = float(geo.sphere_q(dv, c, r))
                lo, hi = 0.0, 1.0
                for _ in range(200):
                    mid = 0.5 * (lo + hi)
                    p = dv + mid * c
                    if np.dot(p, p) >= r * r:
                        lo = mid
                    else:
                        hi = mid
                assert abs(q - 0.5 * (lo + hi)) < 1e-12
                checked += 1
    assert checked > 100
