"""Checkpoint and restart through the C ABI (lbm_state_size / lbm_get_state /
lbm_set_state; the paper restarts one run from another's field, Sec. 2.2.1).

2n steps in one go equal n steps, a save, a restore into a fresh context of
the same configuration and n more steps, bit for bit (fields, particle
state, forces, contact forces), for the dense solver, bounce-back and the
immersed boundary with released moving spheres in contact (FP32 and FP16
storage), the bounce-back and immersed-boundary pipe walls and the D3Q27
pipe solver. A restored context reports the saved fields at once; a blob of
another configuration or a truncated one is rejected and leaves the context
as it was. The blob's populations are the arrays back to back, whatever the
spacing of the device arrays."""
import numpy as np
import pytest

import synth
from paper_1906_05448_amd import lbm
from tests.helpers import gpu_config, gpu_lattice

pytestmark = pytest.mark.gpu


def _snap(g):
    u, rho = g.get_fields()
    out = [u, rho]
    if g.particle_count():
        out += list(g.get_particles()) + list(g.forces())
    return out


def _assert_same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert x.shape == y.shape
        assert np.array_equal(x, y, equal_nan=True)


def _sphere_setup(bc, shape, seed=3):
    spec = synth.hit_spectrum(seed=seed, u_rms=0.04, kcut=10)
    u0 = synth.hit_field(spec, shape)
    # spheres 0 and 1 start in contact; sphere 5 straddles periodic faces
    X = np.array([[10.0, 10.0, 10.0], [19.6, 10.3, 10.0], [30.0, 28.0, 25.0], [12.0, 30.0, 28.0],
                  [36.0, 12.0, 30.0], [46.5, 2.0, 38.7]])
    if bc == 2:
        X[1, 0] = 20.6
    r = np.full(6, 5.0)
    rho_p = np.full(6, 8.0 if bc == 2 else 1.0)

    def setup(g):
        g.set_fields(u0)
        g.set_particles(X, r, rho_p=rho_p, mode=lbm.RELEASE)
    return setup


def _restart_matches(cfg, setup, n1, n2):
    a = gpu_lattice(cfg)
    setup(a)
    a.step(n1)
    saved = _snap(a)
    blob = a.get_state()
    a.step(n2)
    want = _snap(a)
    a.close()
    b = gpu_lattice(cfg)
    b.set_state(blob)
    assert b.step_count == n1
    _assert_same(_snap(b), saved)
    b.step(n2)
    _assert_same(_snap(b), want)
    # restoring into a context that has moved on rewinds it
    b.set_state(blob)
    b.step(n2)
    _assert_same(_snap(b), want)
    b.close()


def test_restart_dense():
    shape = (40, 24, 20)
    cfg = gpu_config(nx=40, ny=24, nz=20, tau=0.6, body_force=(1e-5, 0.0, -5e-6))
    u0 = synth.random_velocity(shape, 0.04, seed=1)
    _restart_matches(cfg, lambda g: g.set_fields(u0), 7, 9)


@pytest.mark.parametrize("bc,store", [(1, 0), (1, 1), (2, 0), (2, 1)])
def test_restart_moving_spheres(bc, store):
    shape = (48, 44, 40)
    cfg = gpu_config(nx=48, ny=44, nz=40, tau=0.55, bc=bc, store=store, ibm_retraction=0.4, max_particles=6,
                     max_radius=5.0, coll_restitution=0.9, coll_tc_steps=8.0)
    _restart_matches(cfg, _sphere_setup(bc, shape), 9, 11)


@pytest.mark.parametrize("bc", [1, 2])
def test_restart_pipe_wall(bc):
    shape = (26, 24, 10)
    R, cx, cy = 9.3, 12.5, 11.7
    cfg = gpu_config(nx=26, ny=24, nz=10, tau=0.8, body_force=(0.0, 0.0, 2e-5), bc=bc, ibb_max_order=1, wall=1,
                     pipe_radius=R, pipe_cx=cx, pipe_cy=cy, ibm_retraction=0.4)
    u0 = synth.pipe_initial_velocity(shape, R, (cx, cy), 0.02, 0.05, seed=2)
    _restart_matches(cfg, lambda g: g.set_fields(u0), 12, 13)


def test_restart_d3q27_pipe():
    shape = (32, 30, 12)
    R, cx, cy = 13.1, 15.5, 14.5
    cfg = gpu_config(nx=32, ny=30, nz=12, tau=0.6, body_force=(0.0, 0.0, 1e-5), bc=1, ibb_max_order=1, wall=1,
                     pipe_radius=R, pipe_cx=cx, pipe_cy=cy, lattice=lbm.LATTICE_D3Q27, tau_bulk=0.9)
    u0 = synth.pipe_initial_velocity(shape, R, (cx, cy), 0.03, 0.05, seed=4)
    _restart_matches(cfg, lambda g: g.set_fields(u0), 6, 6)


def test_rejected_blobs_leave_the_context_unchanged():
    shape = (48, 44, 40)
    cfg = gpu_config(nx=48, ny=44, nz=40, tau=0.55, bc=1, max_particles=6, max_radius=5.0)
    a = gpu_lattice(cfg)
    _sphere_setup(1, shape)(a)
    a.step(3)
    blob = a.get_state()
    other = gpu_lattice(gpu_config(nx=48, ny=44, nz=40, tau=0.56, bc=1, max_particles=6, max_radius=5.0))
    _sphere_setup(1, shape, seed=4)(other)
    other.step(2)
    before = _snap(other)
    with pytest.raises(lbm.LbmError) as e:
        other.set_state(blob)           # another configuration (tau)
    assert e.value.status == -1
    with pytest.raises(lbm.LbmError) as e:
        a.set_state(blob[: len(blob) - 8])  # truncated
    assert e.value.status == -3
    bad = blob.copy()
    bad[:8] = 0                             # not a state blob
    with pytest.raises(lbm.LbmError) as e:
        a.set_state(bad)
    assert e.value.status == -1
    _assert_same(_snap(other), before)
    assert other.step_count == 2
    a.close()
    other.close()


@pytest.mark.parametrize("bc", [1, 2])
def test_rejected_particles_leave_the_context_unchanged(bc):
    """lbm_set_particles validates everything before it changes anything: a
    rejected call (unequal radii with the immersed boundary, a radius above
    the configured maximum, a non-finite position) leaves fields, particles,
    forces and the following steps exactly as without it."""
    shape = (48, 44, 40)
    cfg = gpu_config(nx=48, ny=44, nz=40, tau=0.55, bc=bc, ibm_retraction=0.4 if bc == 2 else 0.0,
                     max_particles=6, max_radius=5.0)
    runs = []
    for reject in (False, True):
        g = gpu_lattice(cfg)
        _sphere_setup(bc, shape)(g)
        g.step(3)
        before = _snap(g)
        if reject:
            X = np.array([[10.0, 10.0, 10.0], [30.0, 28.0, 25.0]])
            bad = [(X, [5.0, 4.0], None), (X, [5.0, 6.0], None), (np.array([[np.nan, 1.0, 1.0]]), [5.0], None)]
            if bc == 1:
                bad = bad[1:]
            for x, r, _ in bad:
                with pytest.raises(lbm.LbmError) as e:
                    g.set_particles(x, r, mode=lbm.RELEASE)
                assert e.value.status == -1
            _assert_same(_snap(g), before)
        g.step(4)
        runs.append(_snap(g))
        g.close()
    _assert_same(runs[1], runs[0])


@pytest.mark.parametrize("store", [0, 1])
def test_blob_populations_are_back_to_back_arrays(store):
    """The blob holds the 19 population arrays of N elements back to back
    right after its header (the device arrays are further apart than their
    length): summed over the arrays, the shifted populations g = f - w
    (FP16: scaled by 2^14) give rho - 1 at every node, against the density
    the context reports."""
    shape = (24, 20, 16)
    N = int(np.prod(shape))
    rng = np.random.default_rng(11)
    u0 = (0.02 * rng.standard_normal((3,) + shape)).astype(np.float32)
    rho0 = (1.0 + 0.01 * rng.standard_normal(shape)).astype(np.float32)
    g = gpu_lattice(gpu_config(nx=shape[0], ny=shape[1], nz=shape[2], tau=0.6, store=store))
    g.set_fields(u0, rho0)
    g.step(3)
    _, rho = g.get_fields()
    blob = g.get_state()
    g.close()
    head = int(np.frombuffer(blob[12:16].tobytes(), np.uint32)[0])
    elem = 4 if store == 0 else 2
    raw = blob[head:head + 19 * N * elem].tobytes()
    if store == 0:
        pops = np.frombuffer(raw, np.float32).astype(np.float64)
    else:
        pops = np.frombuffer(raw, np.float16).astype(np.float64) / 16384.0
    rho_blob = 1.0 + pops.reshape(19, N).sum(axis=0)
    np.testing.assert_allclose(rho_blob, np.asarray(rho, np.float64).reshape(-1), rtol=0, atol=2e-6)
