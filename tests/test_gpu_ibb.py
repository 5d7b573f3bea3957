"""Parity of the HIP interpolated-bounce-back path with the FP64 oracle,
through the C ABI: link geometry bit-exact, fields and particle state
within the FP32 / FP16 tolerances."""
import numpy as np
import pytest

import synth
from oracle.lattice import C as OC
from oracle.sim import RELEASE, SET_RIGID, SET_STATE, Config as OConfig, Sim as OSim
from tests.helpers import gpu_config, gpu_lattice, rel_l2

pytestmark = pytest.mark.gpu

MOTION = {"free": 0, "fixed": 1, "prescribed": 2}


def _pair(shape, tau=0.6, F=(0, 0, 0), store=0, max_order=2, max_np=8, max_r=6.0, **kw):
    o = OSim(OConfig(shape=shape, tau=tau, body_force=tuple(F), bc="ibb", ibb_max_order=max_order, **kw))
    g = gpu_lattice(gpu_config(nx=shape[0], ny=shape[1], nz=shape[2], tau=tau, body_force=tuple(F), bc=1,
                               ibb_max_order=max_order, store=store, max_particles=max_np, max_radius=max_r,
                               **{k: v for k, v in kw.items() if k in ("coll_restitution", "coll_tc_steps")}))
    return o, g


def _oracle_links_sorted(o):
    L = o.state.links
    rows = []
    for (x, y, z), a, p, q, s in zip(L["xf"], L["a"], L["p"], L["q"], L["scheme"]):
        rows.append((int(p), int(x), int(y), int(z), tuple(int(v) for v in OC[a]), np.float32(q), int(s)))
    return sorted(rows, key=lambda r: r[:5])


def _gpu_links_sorted(g):
    L = g.links()
    rows = [(int(p), int(n[0]), int(n[1]), int(n[2]), tuple(int(v) for v in d), np.float32(q), int(s))
            for n, d, p, q, s in zip(L["node"], L["dir"], L["particle"], L["q"], L["scheme"])]
    return sorted(rows, key=lambda r: r[:5])


def test_links_bit_exact_overlapping_and_wrapping_spheres():
    shape = (40, 36, 38)
    X = np.array([[0.37, 17.61, 37.52], [20.2, 18.1, 19.3], [27.9, 18.6, 20.1], [10.5, 33.9, 3.3],
                  [30.01, 5.02, 12.77]])
    r = np.array([5.7, 4.6, 5.2, 3.9, 4.75])
    o, g = _pair(shape, max_r=6.0)
    o.set_particles(X, r=r)
    g.set_particles(X, r)
    lo, lg = _oracle_links_sorted(o), _gpu_links_sorted(g)
    assert len(lo) == len(lg) > 1000
    assert [t[:5] for t in lo] == [t[:5] for t in lg]
    assert [t[6] for t in lo] == [t[6] for t in lg]          # fallback scheme
    assert all(a[5] == b[5] for a, b in zip(lo, lg))         # q, FP64 then rounded to FP32
    assert len({t[6] for t in lo}) >= 2                       # overlaps exercise the fallback chain
    g.close()


@pytest.mark.parametrize("r, shape, X", [
    # small spheres: a few links each, rows of one or two candidates
    (1.6, (24, 20, 22), [[0.4, 10.3, 21.7], [12.2, 9.9, 11.4], [12.9, 13.1, 11.9]]),
    # large spheres: several rounds of rows and link chunks per sphere, a
    # sphere wrapping two faces, two overlapping
    (13.3, (48, 44, 40), [[3.2, 40.7, 3.0], [22.1, 20.3, 19.8], [43.5, 25.0, 23.1]]),
    # the largest radius the immersed boundary admits, in a box just wide enough
    (27.9, (64, 64, 64), [[31.7, 2.4, 60.9]]),
])
def test_links_bit_exact_small_and_large_spheres(r, shape, X):
    """Link sets, q and schemes bit-exact against the oracle at radii that
    take the link build's row spans and LDS planes to their extremes."""
    X = np.asarray(X, float)
    rr = np.full(len(X), r)
    o, g = _pair(shape, max_np=len(X), max_r=r)
    o.set_particles(X, r=rr)
    g.set_particles(X, rr)
    lo, lg = _oracle_links_sorted(o), _gpu_links_sorted(g)
    assert len(lo) == len(lg) > 0
    assert [t[:5] for t in lo] == [t[:5] for t in lg]
    assert [t[6] for t in lo] == [t[6] for t in lg]
    assert all(a[5] == b[5] for a, b in zip(lo, lg))
    solid_o = int((o.state.owner >= 0).sum())
    assert g.geometry_counts()[0] == solid_o
    g.close()


@pytest.mark.parametrize("store", [0, 1])
def test_fixed_sphere_body_force_500_steps(store):
    """Fixed sphere r = 4.5 at the centre of a 32^3 box driven by g = 1e-6,
    quadratic IBB, 500 steps from rest (the plain-method drag case)."""
    shape = (32, 32, 32)
    F = (1e-6, 0.0, 0.0)
    o, g = _pair(shape, tau=0.6, F=F, store=store, max_np=1, max_r=4.5)
    o.set_particles([[16.0, 16.0, 16.0]], r=[4.5], motion="fixed")
    g.set_particles([[16.0, 16.0, 16.0]], [4.5], motion=MOTION["fixed"])
    for chunk in (1, 9, 90, 400):
        o.step(chunk)
        g.step(chunk)
        fluid = o.fluid_mask()
        ug, _ = g.get_fields()
        uo, _ = o.fields()
        tol = 1e-5 if store == 0 else 2e-3
        assert rel_l2(ug, uo, fluid) < tol, o.state.step
        Fg, Tg, _ = g.forces()
        Fo, To, _ = o.forces()
        # from rest the first step's link forces cancel to round-off
        assert abs(Fg[0, 0] - Fo[0, 0]) <= (1e-5 if store == 0 else 3e-3) * abs(Fo[0, 0]) + 1e-12
    g.close()


@pytest.mark.parametrize("store", [0, 1])
def test_moving_spheres_release_contact_refill(store):
    """Freely moving neutrally buoyant spheres released into a seeded
    turbulence field: refill, cover/uncover momentum, contact forces."""
    shape = (48, 44, 40)
    spec = synth.hit_spectrum(seed=3, u_rms=0.04, kcut=10)
    u0 = synth.hit_field(spec, shape)
    # spheres 0 and 1 start in contact (gap -0.4); sphere 5 straddles three
    # periodic faces; all other gaps exceed 6 lattice units
    X = np.array([[10.0, 10.0, 10.0], [19.6, 10.3, 10.0], [30.0, 28.0, 25.0], [12.0, 30.0, 28.0],
                  [36.0, 12.0, 30.0], [46.5, 2.0, 38.7]])
    r = np.full(6, 5.0)
    o, g = _pair(shape, tau=0.55, store=store, max_np=6, max_r=5.0, coll_restitution=0.9, coll_tc_steps=8.0)
    o.set_fields(u0)
    g.set_fields(u0)
    o.set_particles(X, r=r, mode=RELEASE)
    g.set_particles(X, r, mode=1)
    Xg, Ug, _ = g.get_particles()
    Xo, Uo = o.state.P.X, o.state.P.U
    assert np.abs(Xg - Xo).max() < 1e-12
    assert np.abs(Ug - Uo).max() < (1e-6 if store == 0 else 2e-3) * np.abs(Uo).max()
    moved = 0
    for _ in range(6):
        o.step(5)
        g.step(5)
        moved += o.state.extra["uncovered"]
        fluid = o.fluid_mask()
        ug, _ = g.get_fields()
        uo, _ = o.fields()
        tol = 1e-5 if store == 0 else 2e-3
        assert rel_l2(ug, uo, fluid) < tol, o.state.step
        Xg, Ug, Wg = g.get_particles()
        P = o.state.P
        assert np.abs(Xg - P.X).max() < (1e-6 if store == 0 else 2e-4)
        assert rel_l2(Ug, P.U) < (1e-4 if store == 0 else 1e-2)
        assert rel_l2(Wg, P.Om) < (1e-3 if store == 0 else 5e-2)
        Fg, Tg, Fcg = g.forces()
        Fo, To, Fco = o.forces()
        assert rel_l2(Fg, Fo) < (1e-4 if store == 0 else 2e-2)
        assert rel_l2(Tg, To) < (1e-3 if store == 0 else 5e-2)
        assert np.abs(Fco).max() == 0 or rel_l2(Fcg, Fco) < (1e-6 if store == 0 else 1e-3)
    assert np.abs(o.state.F_c).max() > 0 or moved > 0
    assert np.abs(o.state.P.Om).max() > 1e-6  # the spheres spin up
    g.close()


@pytest.mark.parametrize("store", [0, 1])
def test_r8_spheres_release_quadratic_ibb(store):
    """Radius 8, the production spheres: three released spheres, two of them
    in near contact (gap 0.6: their links fall back from quadratic), one
    across periodic faces; density ratio 4; fields, particle state, forces and
    torques against the oracle."""
    shape = (56, 48, 44)
    spec = synth.hit_spectrum(seed=7, u_rms=0.03, kcut=8)
    u0 = synth.hit_field(spec, shape)
    X = np.array([[15.3, 20.2, 21.7], [31.8, 21.1, 22.3], [50.6, 40.9, 6.4]])
    r = np.full(3, 8.0)
    rho_p = np.full(3, 4.0)
    o, g = _pair(shape, tau=0.52, store=store, max_np=3, max_r=8.0)
    o.set_fields(u0)
    g.set_fields(u0)
    o.set_particles(X, r=r, rho_p=rho_p, mode=RELEASE)
    g.set_particles(X, r, rho_p=rho_p, mode=1)
    lo, lg = _oracle_links_sorted(o), _gpu_links_sorted(g)
    assert [t[:5] for t in lo] == [t[:5] for t in lg] and len({t[6] for t in lo}) >= 2
    tol = 1e-5 if store == 0 else 2e-3
    for chunk in (1, 4, 10):
        o.step(chunk)
        g.step(chunk)
        fluid = o.fluid_mask()
        ug, _ = g.get_fields()
        uo, _ = o.fields()
        assert rel_l2(ug, uo, fluid) < tol, o.state.step
        Xg, Ug, Wg = g.get_particles()
        P = o.state.P
        assert np.abs(Xg - P.X).max() < (1e-6 if store == 0 else 2e-4)
        assert rel_l2(Ug, P.U) < (1e-4 if store == 0 else 1e-2)
        assert rel_l2(Wg, P.Om) < (1e-3 if store == 0 else 5e-2)
        Fg, Tg, _ = g.forces()
        Fo, To, _ = o.forces()
        assert rel_l2(Fg, Fo) < (1e-4 if store == 0 else 2e-2)
        assert rel_l2(Tg, To) < (1e-3 if store == 0 else 5e-2)
    g.close()


@pytest.mark.parametrize("store", [0, 1])
def test_release_velocity_large_sphere(store):
    """The release velocity (Sec. 3.1: the fluid velocity averaged over the
    particle volume with the cells' solid fractions) of a radius-20 sphere
    across a periodic face: about 37 000 cells within r + sqrt(3)/2, so the
    Kempe-weighted average takes about ten rounds of its LDS cell list."""
    shape = (48, 48, 48)
    spec = synth.hit_spectrum(seed=4, u_rms=0.03, kcut=8)
    u0 = synth.hit_field(spec, shape)
    X = np.array([[23.7, 24.2, 1.9]])
    o, g = _pair(shape, tau=0.55, store=store, max_np=1, max_r=20.0)
    o.set_fields(u0)
    g.set_fields(u0)
    o.set_particles(X, r=[20.0], rho_p=[2.0], mode=RELEASE)
    g.set_particles(X, [20.0], rho_p=[2.0], mode=1)
    _, Ug, Wg = g.get_particles()
    assert np.abs(o.state.P.U).max() > 1e-4
    assert rel_l2(Ug, o.state.P.U) < (1e-6 if store == 0 else 2e-3)
    assert np.all(Wg == 0.0)
    g.close()


def test_overlap_latch():
    """Soft-sphere contact (Sec. 3.1) keeps spheres apart; an overlap deeper
    than half a radius is reported as LBM_E_OVERLAP by the next syncing call
    and the latch clears; a shallow one is not an error."""
    from paper_1906_05448_amd import lbm
    shape = (40, 32, 32)
    g = gpu_lattice(gpu_config(nx=40, ny=32, nz=32, tau=0.6, bc=1, max_particles=2, max_radius=5.0))
    g.set_particles([[12.0, 16.0, 16.0], [21.0, 16.0, 16.0]], [5.0, 5.0])  # overlap 1 < 2.5
    g.step(1)
    g.sync()
    g.set_particles([[12.0, 16.0, 16.0], [19.0, 16.0, 16.0]], [5.0, 5.0])  # overlap 3 > 2.5
    g.step(1)
    with pytest.raises(lbm.LbmError) as e:
        g.sync()
    assert e.value.status == -6
    g.sync()
    g.close()


def test_comoving_sphere_stays_uniform_on_gpu():
    shape = (24, 20, 22)
    U = np.array([0.021, -0.013, 0.008])
    o, g = _pair(shape, tau=0.7, max_np=1, max_r=4.0)
    u0 = np.broadcast_to(U[:, None, None, None], (3, 22, 20, 24))
    g.set_particles([[11.3, 9.9, 10.6]], [3.4], u=[U], motion=MOTION["prescribed"])
    g.set_fields(u0)
    g.step(80)
    ug, rg = g.get_fields()
    X, _, _ = g.get_particles()
    owner = __import__("oracle.geometry", fromlist=["owner_map"]).owner_map(shape, X, np.array([3.4]))
    fluid = owner == -1
    assert np.abs(ug[:, fluid] - U[:, None]).max() < 2e-6
    assert np.abs(rg[fluid] - 1).max() < 2e-6
    g.close()


def test_pipe_wall_linear_ibb():
    """Static pipe wall along z (linear IBB, ray-cylinder q), body-force
    driven, FP32 vs FP64."""
    shape = (24, 24, 8)
    F = (0.0, 0.0, 2e-5)
    kw = dict(wall="pipe_z", pipe_radius=9.3, pipe_cx=11.5, pipe_cy=11.7)
    o = OSim(OConfig(shape=shape, tau=0.8, body_force=F, bc="ibb", ibb_max_order=1, **kw))
    g = gpu_lattice(gpu_config(nx=24, ny=24, nz=8, tau=0.8, body_force=F, bc=1, ibb_max_order=1, wall=1,
                               pipe_radius=9.3, pipe_cx=11.5, pipe_cy=11.7))
    lo, lg = _oracle_links_sorted(o), _gpu_links_sorted(g)
    assert [t[1:5] for t in lo] == [t[1:5] for t in lg]
    assert all(a[5] == b[5] and a[6] == b[6] for a, b in zip(lo, lg))
    o.step(200)
    g.step(200)
    ug, _ = g.get_fields()
    uo, _ = o.fields()
    assert rel_l2(ug, uo, o.fluid_mask()) < 1e-5
    g.close()


@pytest.mark.parametrize("store", [0, 1])
def test_prescribed_spheres_cross_periodic_faces(store):
    """Two spheres with prescribed velocity and spin cross periodic faces
    (x and z for one, y for the other) while they move: the wrapped
    positions, the refill of uncovered nodes and the cover/uncover momentum
    must follow the oracle across the wrap."""
    shape = (28, 26, 30)
    X = np.array([[0.6, 12.0, 29.5], [14.0, 25.4, 15.0]])
    U = np.array([[-0.06, 0.01, 0.05], [0.02, 0.07, -0.01]])
    W = np.array([[0.0, 0.004, -0.003], [0.002, 0.0, 0.005]])
    r = np.array([4.3, 3.8])
    o, g = _pair(shape, tau=0.6, store=store, max_np=2, max_r=4.5)
    spec = synth.hit_spectrum(seed=5, u_rms=0.02, kcut=6)
    u0 = synth.hit_field(spec, shape)
    o.set_fields(u0)
    g.set_fields(u0)
    o.set_particles(X, U=U, Om=W, r=r, mode=SET_RIGID, motion="prescribed")
    g.set_particles(X, r, u=U, omega=W, mode=2, motion=MOTION["prescribed"])
    uncovered = 0
    for _ in range(4):
        o.step(6)
        g.step(6)
        uncovered += o.state.extra["uncovered"]
        Xg, _, _ = g.get_particles()
        assert np.abs(Xg - o.state.P.X).max() < 1e-9
        ug, _ = g.get_fields()
        uo, _ = o.fields()
        tol = 1e-5 if store == 0 else 2e-3
        assert rel_l2(ug, uo, o.fluid_mask()) < tol, o.state.step
        Fg, _, _ = g.forces()
        Fo, _, _ = o.forces()
        assert rel_l2(Fg, Fo) < (1e-4 if store == 0 else 2e-2)
    # both spheres wrapped at least once
    Xf = o.state.P.X
    assert Xf[0, 0] > 20 and Xf[0, 2] < 5 and Xf[1, 1] < 5
    assert uncovered > 0
    g.close()


def test_prescribed_large_sphere_fast_motion():
    """A large sphere (r = 11.7) moving 0.12 nodes a step with spin across a
    periodic face, next to a smaller one moving the other way: many nodes
    change side every step, so the owner passes and the refill lists are
    exercised at full width; solid counts exact, fields and forces at the
    FP32 bar."""
    shape = (40, 36, 34)
    X = np.array([[38.9, 17.2, 16.1], [20.3, 8.9, 20.4]])
    U = np.array([[0.12, -0.03, 0.02], [-0.05, 0.08, 0.0]])
    W = np.array([[0.003, -0.002, 0.004], [0.0, 0.006, -0.002]])
    r = np.array([11.7, 5.2])
    o, g = _pair(shape, tau=0.6, store=0, max_np=2, max_r=11.7)
    spec = synth.hit_spectrum(seed=9, u_rms=0.02, kcut=6)
    u0 = synth.hit_field(spec, shape)
    o.set_fields(u0)
    g.set_fields(u0)
    o.set_particles(X, U=U, Om=W, r=r, mode=SET_RIGID, motion="prescribed")
    g.set_particles(X, r, u=U, omega=W, mode=2, motion=MOTION["prescribed"])
    uncovered = 0
    for _ in range(4):
        o.step(5)
        g.step(5)
        uncovered += o.state.extra["uncovered"]
        assert g.geometry_counts()[0] == int((o.state.owner >= 0).sum())
        ug, _ = g.get_fields()
        uo, _ = o.fields()
        assert rel_l2(ug, uo, o.fluid_mask()) < 1e-5, o.state.step
        Fg, _, _ = g.forces()
        Fo, _, _ = o.forces()
        assert rel_l2(Fg, Fo) < 1e-4
    assert o.state.P.X[0, 0] < 10  # crossed the x face
    assert uncovered > 200
    g.close()


def _crowded_sphere(centre, R, r, n, overlap):
    """A sphere of radius R touched by n spheres of radius r, centres on a
    Fibonacci lattice at distance R + r - overlap."""
    k = np.arange(n) + 0.5
    phi = np.arccos(1.0 - 2.0 * k / n)
    theta = np.pi * (1.0 + 5.0 ** 0.5) * k
    d = np.stack([np.cos(theta) * np.sin(phi), np.sin(theta) * np.sin(phi), np.cos(phi)], axis=1)
    X = np.vstack([centre, np.asarray(centre) + (R + r - overlap) * d])
    rad = np.concatenate([[R], np.full(n, r)])
    return X, rad


@pytest.mark.parametrize("side", [40, 52])
def test_contact_forces_many_partners(side):
    """One sphere touched by 70 others, more partners than one particle's
    collected list holds, on contact grids of one (40^3) and two (52^3)
    cells per axis. Contact forces follow the soft-sphere law of Sec. 3.1
    summed in index order; pair forces cancel (Newton's third law)."""
    c = side / 2.0
    X, rad = _crowded_sphere((c, c, c), 12.0, 2.0, 70, 0.3)
    dmin = min(np.linalg.norm(X[1:] - X[i], axis=1)[i:].min() for i in range(1, 70))
    assert dmin > 2 * 2.0  # only the central sphere is in contact
    U = np.random.default_rng(11).normal(scale=0.01, size=X.shape)
    shape = (side, side, side)
    o, g = _pair(shape, tau=0.6, max_np=71, max_r=12.0, coll_restitution=0.9, coll_tc_steps=8.0)
    o.set_particles(X, U=U, r=rad)
    g.set_particles(X, rad, u=U)
    o.step(1)
    g.step(1)
    _, _, Fcg = g.forces()
    Fco = o.state.F_c
    assert np.abs(Fco[0]).max() > 0 and np.all(np.abs(Fco[1:]).max(axis=1) > 0)
    assert np.abs(Fcg - Fco).max() <= 1e-12 * np.abs(Fco).max()
    assert np.abs(Fcg.sum(axis=0)).max() <= 1e-12 * np.abs(Fcg).max()
    g.close()
