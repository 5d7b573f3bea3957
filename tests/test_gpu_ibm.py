"""Parity of the HIP immersed-boundary path (multi-direct forcing, Peskin
delta, Kempe inner inertia) with the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import synth
from oracle.sim import RELEASE, Config as OConfig, Sim as OSim
from tests.helpers import gpu_config, gpu_lattice, rel_l2

pytestmark = pytest.mark.gpu

MOTION = {"free": 0, "fixed": 1, "prescribed": 2}


def _pair(shape, tau=0.6, F=(0, 0, 0), store=0, rd=0.0, iters=2, max_np=8, max_r=6.0, **kw):
    o = OSim(OConfig(shape=shape, tau=tau, body_force=tuple(F), bc="ibm", ibm_retraction=rd, ibm_iters=iters, **kw))
    g = gpu_lattice(gpu_config(nx=shape[0], ny=shape[1], nz=shape[2], tau=tau, body_force=tuple(F), bc=2,
                               ibm_retraction=rd, ibm_iters=iters, store=store, max_particles=max_np,
                               max_radius=max_r, **kw))
    return o, g


@pytest.mark.parametrize("store,rd", [(0, 0.0), (0, 0.4), (1, 0.4)])
def test_fixed_sphere_body_force_500_steps(store, rd):
    """Fixed sphere r = 4.5 at the centre of a 32^3 box, g = 1e-6, 500 steps
    from rest, Uhlmann (r_d = 0) and Breugem (r_d = 0.4) markers."""
    shape = (32, 32, 32)
    F = (1e-6, 0.0, 0.0)
    o, g = _pair(shape, tau=0.6, F=F, store=store, rd=rd, max_np=1, max_r=4.5)
    o.set_particles([[16.0, 16.0, 16.0]], r=[4.5], motion="fixed")
    g.set_particles([[16.0, 16.0, 16.0]], [4.5], motion=MOTION["fixed"])
    tol = 1e-5 if store == 0 else 2e-3
    for chunk in (1, 9, 90, 400):
        o.step(chunk)
        g.step(chunk)
        ug, _ = g.get_fields()
        uo, _ = o.fields()
        assert rel_l2(ug, uo) < tol, o.state.step
        Fg, _, _ = g.forces()
        Fo, _, _ = o.forces()
        assert abs(Fg[0, 0] - Fo[0, 0]) <= (1e-4 if store == 0 else 5e-3) * abs(Fo[0, 0]) + 1e-12
    g.close()


@pytest.mark.parametrize("store", [0, 1])
def test_moving_spheres_release_ibm(store):
    """Released spheres in a seeded turbulence field: forcing passes, Kempe
    inner inertia, moving supports (IBM-B). Density ratio 8: the explicit
    inner-inertia coupling is stable when the diffuse shell outside a sphere
    is light compared with the sphere (about 5 w / (rho_p r) < 1 for
    rotation, w ~ 3.5 cells); at rho_p = 1 and r = 5 it diverges."""
    shape = (48, 44, 40)
    spec = synth.hit_spectrum(seed=3, u_rms=0.04, kcut=10)
    u0 = synth.hit_field(spec, shape)
    X = np.array([[10.0, 10.0, 10.0], [20.6, 10.3, 10.0], [30.0, 28.0, 25.0], [12.0, 30.0, 28.0],
                  [36.0, 12.0, 30.0], [46.5, 2.0, 38.7]])
    r = np.full(6, 5.0)
    rho_p = np.full(6, 8.0)
    o, g = _pair(shape, tau=0.55, store=store, rd=0.4, max_np=6, max_r=5.0, coll_restitution=0.9,
                 coll_tc_steps=8.0)
    o.set_fields(u0)
    g.set_fields(u0)
    o.set_particles(X, r=r, rho_p=rho_p, mode=RELEASE)
    g.set_particles(X, r, rho_p=rho_p, mode=1)
    Xg, Ug, _ = g.get_particles()
    assert np.abs(Ug - o.state.P.U).max() < (1e-6 if store == 0 else 2e-3) * np.abs(o.state.P.U).max()
    tol = 1e-5 if store == 0 else 2e-3
    for _ in range(6):
        o.step(5)
        g.step(5)
        ug, _ = g.get_fields()
        uo, _ = o.fields()
        assert rel_l2(ug, uo) < tol, o.state.step
        Xg, Ug, Wg = g.get_particles()
        P = o.state.P
        assert np.abs(Xg - P.X).max() < (1e-6 if store == 0 else 2e-4)
        assert rel_l2(Ug, P.U) < (1e-4 if store == 0 else 1e-2)
        assert rel_l2(Wg, P.Om) < (1e-3 if store == 0 else 5e-2)
        Fg, Tg, _ = g.forces()
        Fo, To, _ = o.forces()
        assert rel_l2(Fg, Fo) < (1e-4 if store == 0 else 2e-2)
        assert rel_l2(Tg, To) < (1e-3 if store == 0 else 5e-2)
    assert np.abs(o.state.P.Om).max() > 1e-6  # the spheres spin up
    g.close()


@pytest.mark.parametrize("store,rd", [(0, 0.0), (0, 0.4), (1, 0.0), (1, 0.4)])
def test_r8_spheres_sharing_support(store, rd):
    """Radius 8, the production spheres: the forcing support of one sphere
    (about 4 500 nodes at r_d = 0, 4 100 at r_d = 0.4) takes one or two
    staging rounds of 4 096 nodes in the pass kernel. Three released spheres, two of them 2 spacings apart so that
    their supports share nodes, one across a periodic face; density ratio 4
    as in the paper's particle-laden case."""
    shape = (56, 48, 44)
    spec = synth.hit_spectrum(seed=7, u_rms=0.03, kcut=8)
    u0 = synth.hit_field(spec, shape)
    X = np.array([[15.3, 20.2, 21.7], [33.4, 21.1, 22.3], [50.6, 40.9, 6.4]])
    r = np.full(3, 8.0)
    rho_p = np.full(3, 4.0)
    o, g = _pair(shape, tau=0.52, store=store, rd=rd, max_np=3, max_r=8.0)
    o.set_fields(u0)
    g.set_fields(u0)
    o.set_particles(X, r=r, rho_p=rho_p, mode=RELEASE)
    g.set_particles(X, r, rho_p=rho_p, mode=1)
    tol = 1e-5 if store == 0 else 2e-3
    for chunk in (1, 4, 10):
        o.step(chunk)
        g.step(chunk)
        ug, _ = g.get_fields()
        uo, _ = o.fields()
        assert rel_l2(ug, uo) < tol, o.state.step
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
def test_r10_spheres_two_markers_per_thread(store):
    """Radius 10 at r_d = 0.4: 1159 markers per sphere, so the pass kernel
    takes two markers per thread (one 1024-thread workgroup per compute
    unit), the forcing support of a sphere (about 6 500 nodes) two staging
    rounds, and the Kempe integral (about 5 400 cells within r + sqrt(3)/2)
    two rounds of its LDS cell list. Two released spheres whose supports
    share nodes, one of them across a periodic face."""
    shape = (52, 48, 44)
    spec = synth.hit_spectrum(seed=12, u_rms=0.03, kcut=8)
    u0 = synth.hit_field(spec, shape)
    X = np.array([[5.3, 22.2, 20.9], [27.4, 23.1, 22.6]])
    r = np.full(2, 10.0)
    rho_p = np.full(2, 4.0)
    o, g = _pair(shape, tau=0.52, store=store, rd=0.4, max_np=2, max_r=10.0)
    o.set_fields(u0)
    g.set_fields(u0)
    o.set_particles(X, r=r, rho_p=rho_p, mode=RELEASE)
    g.set_particles(X, r, rho_p=rho_p, mode=1)
    tol = 1e-5 if store == 0 else 2e-3
    for chunk in (1, 4, 10):
        o.step(chunk)
        g.step(chunk)
        ug, _ = g.get_fields()
        uo, _ = o.fields()
        assert rel_l2(ug, uo) < tol, o.state.step
        Xg, Ug, Wg = g.get_particles()
        P = o.state.P
        assert np.abs(Xg - P.X).max() < (1e-6 if store == 0 else 2e-4)
        assert rel_l2(Ug, P.U) < (1e-4 if store == 0 else 1e-2)
        assert rel_l2(Wg, P.Om) < (1e-3 if store == 0 else 5e-2)
        Fg, Tg, _ = g.forces()
        Fo, To, _ = o.forces()
        assert rel_l2(Fg, Fo) < (1e-4 if store == 0 else 2e-2)
        assert rel_l2(Tg, To) < (1e-3 if store == 0 else 5e-2)
    support, shared = g.ibm_support()
    assert support > 2 * 6000 and shared > 0
    g.close()


def test_many_spheres_jacobi_passes_reproducible():
    """More spheres than the device runs at once (1200 of radius 3.5 in a
    112^3 box, supports overlapping everywhere): every marker of a forcing
    pass reads the velocity of the end of the previous pass (Jacobi across
    spheres, as the oracle), whichever order the workgroups run in, and the
    shared-node sums are exact, so two runs agree bit for bit and both match
    the FP64 oracle."""
    shape = (112, 112, 112)
    n, r = 1200, 3.5
    X = synth.random_spheres(n, shape, 2 * r + 1.0, seed=21)
    rng = np.random.default_rng(5)
    U = rng.normal(scale=0.01, size=(n, 3))
    W = rng.normal(scale=0.002, size=(n, 3))
    spec = synth.hit_spectrum(seed=8, u_rms=0.03, kcut=12)
    u0 = synth.hit_field(spec, shape)
    runs = []
    for _ in range(2):
        g = gpu_lattice(gpu_config(nx=112, ny=112, nz=112, tau=0.55, bc=2, max_particles=n, max_radius=r))
        g.set_fields(u0)
        g.set_particles(X, np.full(n, r), u=U, omega=W, rho_p=np.full(n, 8.0))
        g.step(3)
        runs.append([*g.get_fields(), *g.get_particles(), *g.forces()])
        g.close()
    for a, b in zip(*runs):
        assert np.array_equal(a, b)
    o = OSim(OConfig(shape=shape, tau=0.55, bc="ibm"))
    o.set_fields(u0)
    o.set_particles(X, U=U, Om=W, r=np.full(n, r), rho_p=np.full(n, 8.0))
    o.step(3)
    uo, _ = o.fields()
    ug = runs[0][0]
    assert rel_l2(ug, uo) < 1e-5
    Fo, To, _ = o.forces()
    assert rel_l2(runs[0][5], Fo) < 1e-4
    assert rel_l2(runs[0][6], To) < 1e-3
    assert rel_l2(runs[0][3], o.state.P.U) < 1e-4


def test_comoving_sphere_ibm_keeps_uniform_flow():
    shape = (24, 20, 22)
    U = np.array([0.021, -0.013, 0.008])
    o, g = _pair(shape, tau=0.7, max_np=1, max_r=4.0)
    g.set_fields(np.broadcast_to(U[:, None, None, None], (3, 22, 20, 24)))
    g.set_particles([[11.3, 9.9, 10.6]], [3.4], u=[U], motion=MOTION["prescribed"])
    g.step(60)
    ug, rg = g.get_fields()
    assert np.abs(ug - U[:, None, None, None]).max() < 2e-6
    assert np.abs(rg - 1).max() < 2e-6
    g.close()


@pytest.mark.parametrize("store,rd", [(0, 0.0), (0, 0.4), (1, 0.4)])
def test_pipe_wall_ibm(store, rd):
    """Immersed-boundary pipe wall (static marker rings at every integer z,
    Uhlmann r_d = 0 and Breugem r_d = 0.4), body-force driven from a
    perturbed parabolic profile, 200 steps, against the FP64 oracle; the
    body force acts inside the pipe only."""
    from oracle import stats as ostats
    shape = (26, 24, 10)
    R, cx, cy = 9.3, 12.5, 11.7
    F = (0.0, 0.0, 2e-5)
    kw = dict(wall="pipe_z", pipe_radius=R, pipe_cx=cx, pipe_cy=cy)
    o = OSim(OConfig(shape=shape, tau=0.8, body_force=F, bc="ibm", ibm_retraction=rd, **kw))
    g = gpu_lattice(gpu_config(nx=26, ny=24, nz=10, tau=0.8, body_force=F, bc=2, ibm_retraction=rd, store=store,
                               wall=1, pipe_radius=R, pipe_cx=cx, pipe_cy=cy))
    u0 = synth.pipe_initial_velocity(shape, R, (cx, cy), 0.02, 0.05, seed=2)
    o.set_fields(u0)
    g.set_fields(u0)
    tol = 1e-5 if store == 0 else 2e-3
    for chunk in (1, 9, 90, 100):
        o.step(chunk)
        g.step(chunk)
        ug, _ = g.get_fields()
        uo, ro = o.fields()
        assert rel_l2(ug, uo) < tol, o.state.step
    so = ostats.statistics(uo, ro, (0.8 - 0.5) / 3, shape, pipe=(R, cx, cy), nbins=0)
    sg = g.stats(nbins=0)
    assert abs(sg["bulk_u"] - so["bulk_u"]) < tol * abs(so["bulk_u"])
    assert sg["n_fluid"] == so["n_fluid"]
    g.close()
