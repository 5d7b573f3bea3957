"""Parity of the HIP dense path (fused pull-stream + MRT + Guo) with the
FP64 oracle, through the C ABI.

Tolerances (relative L2 of the velocity over all nodes): 1e-5 with FP32
storage, 2e-3 with FP16 shifted storage."""
import numpy as np
import pytest

import synth
from oracle import collide as col
from oracle.lattice import C as OC
from oracle.sim import Config as OConfig, Sim as OSim
from tests.helpers import gpu_config, gpu_lattice, rel_l2

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 2e-3}


def _run_pair(shape, tau, F, u0, rho0, steps, store):
    o = OSim(OConfig(shape=shape, tau=tau, body_force=tuple(F)))
    o.set_fields(u0, rho0)
    o.step(steps)
    g = gpu_lattice(gpu_config(nx=shape[0], ny=shape[1], nz=shape[2], tau=tau, body_force=tuple(F), store=store))
    g.set_fields(u0, rho0)
    g.step(steps)
    ug, rg = g.get_fields()
    g.close()
    uo, ro = o.fields()
    return ug, rg, uo, ro


@pytest.mark.parametrize("store", [0, 1])
def test_dense_ragged_tiles(store):
    # 70 x 13 x 9 spans two 64-wide tiles with a ragged x tail and a ragged
    # y tail of the 4-row tiles.
    shape = (70, 13, 9)
    F = (1e-5, -2e-5, 5e-6)
    u0 = synth.random_velocity(shape, 0.05, seed=11)
    r0 = synth.random_density(shape, 0.01, seed=12)
    ug, rg, uo, ro = _run_pair(shape, 0.6, F, u0, r0, 20, store)
    assert rel_l2(ug, uo) < TOL[store]
    assert rel_l2(rg - 1, ro - 1) < 50 * TOL[store]


@pytest.mark.parametrize("store", [0, 1])
def test_dense_hit_field_100_steps(store):
    shape = (48, 48, 48)
    spec = synth.hit_spectrum(seed=0, u_rms=0.03, kcut=12)
    u0 = synth.hit_field(spec, shape)
    ug, rg, uo, ro = _run_pair(shape, 0.52, (0, 0, 0), u0, None, 100, store)
    assert rel_l2(ug, uo) < TOL[store]


@pytest.mark.parametrize("store", [0, 1])
def test_dense_minimum_box(store):
    shape = (4, 4, 4)
    u0 = synth.random_velocity(shape, 0.03, seed=3)
    ug, rg, uo, ro = _run_pair(shape, 0.9, (1e-4, 0, 0), u0, None, 10, store)
    assert rel_l2(ug, uo) < TOL[store]


@pytest.mark.parametrize("shape", [(71, 6, 5), (130, 5, 4), (6, 6, 5), (128, 4, 4), (512, 5, 4), (1024, 4, 4),
                                   (1536, 4, 5)])
def test_dense_fp16_row_lengths(shape):
    # FP16 storage over row lengths around the 64-node tile: an odd row (71),
    # one node past two tiles (130), a row shorter than a wavefront (6) and
    # exactly two tiles (128); a row of 512 nodes takes the kernel whose
    # workgroup holds the whole row and passes the segment ends between its
    # wavefronts (periodic inside it), rows of 1024 and 1536 the tiled one;
    # the x-wrap of the shifted directions is exercised at both ends of every
    # row.
    F = (2e-5, 1e-5, -1e-5)
    u0 = synth.random_velocity(shape, 0.05, seed=21)
    r0 = synth.random_density(shape, 0.01, seed=22)
    ug, rg, uo, ro = _run_pair(shape, 0.6, F, u0, r0, 15, 1)
    assert rel_l2(ug, uo) < TOL[1]
    assert rel_l2(rg - 1, ro - 1) < 50 * TOL[1]


def test_dense_zero_steps_returns_initial_state():
    shape = (16, 8, 8)
    u0 = synth.random_velocity(shape, 0.03, seed=4)
    r0 = synth.random_density(shape, 0.01, seed=5)
    ug, rg, uo, ro = _run_pair(shape, 0.7, (0, 0, 0), u0, r0, 0, 0)
    assert rel_l2(ug, uo) < 1e-6 and np.abs(rg - ro).max() < 1e-6


@pytest.mark.parametrize("store", [0, 1])
def test_dense_full_size_sampled(store):
    """512^3 (the benchmark lattice), one step from the seeded turbulence
    field; the oracle recomputes sampled nodes one by one from the same
    field evaluated pointwise."""
    n = 512
    shape = (n, n, n)
    tau = 0.52
    spec = synth.hit_spectrum(seed=0, u_rms=0.03)
    g = gpu_lattice(gpu_config(nx=n, ny=n, nz=n, tau=tau, store=store))
    import torch
    u0 = torch.from_numpy(synth.hit_field(spec, shape, dtype=np.float32)).cuda()
    g.set_fields_device(u0)
    g.step(1)
    ug = torch.empty_like(u0)
    rg = torch.empty(u0.shape[1:], dtype=torch.float32, device=u0.device)
    g.get_fields_device(ug, rg)
    g.sync()
    rng = np.random.default_rng(7)
    pts = rng.integers(0, n, size=(96, 3))
    pts[:8] = [[0, 0, 0], [n - 1, n - 1, n - 1], [0, n - 1, 5], [n - 1, 0, 9], [63, 64, 1], [64, 3, n - 1],
               [511, 255, 0], [1, 1, 1]]
    o = OConfig(shape=shape, tau=tau)
    s = o.rates()
    errs = []
    for x, y, z in pts:
        src = np.array([((x - OC[i, 0]) % n, (y - OC[i, 1]) % n, (z - OC[i, 2]) % n) for i in range(19)])
        uu = synth.hit_field_at(spec, shape, src)                       # (19, 3)
        f = np.array([col.equilibrium(1.0, uu[i])[i] for i in range(19)]).reshape(19, 1, 1, 1)
        _, rho, u = col.collide(f, np.zeros((3, 1, 1, 1)), s)
        got = ug[:, z, y, x].cpu().numpy().astype(np.float64)
        errs.append(np.linalg.norm(got - u.ravel()) / max(np.linalg.norm(u.ravel()), 1e-3))
        assert abs(float(rg[z, y, x]) - rho.item()) < (1e-6 if store == 0 else 1e-3)
    g.close()
    assert np.sqrt(np.mean(np.square(errs))) < TOL[store]


@pytest.mark.parametrize("store,nx", [(0, 8), (1, 8), (1, 9)])
def test_instability_is_reported(store, nx):
    # both stream-collide kernels latch it: FP32 / odd-row FP16 (one node per
    # lane) and even-row FP16 (rows staged through LDS)
    from paper_1906_05448_amd import lbm
    g = gpu_lattice(gpu_config(nx=nx, ny=8, nz=8, tau=0.6, store=store))
    u = np.zeros((3, 8, 8, nx))
    u[0] = 0.4                      # above the |u| < 0.35 guard
    g.set_fields(u)
    g.step(1)
    with pytest.raises(lbm.LbmError) as ei:
        g.sync()
    assert ei.value.status == -5
    g.sync()                        # the latch clears once reported
    g.close()
