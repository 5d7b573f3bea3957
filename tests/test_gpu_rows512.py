"""Rows of 512 nodes take the stream-collide kernels whose workgroup holds
the whole row (FP32 and FP16 storage) and passes the segment ends between
its wavefronts; longer rows (1024, 1536) take the tiled kernels. Parity
with the FP64 oracle on thin boxes: the plain update, and moving spheres
with bounce-back and with the immersed boundary (whose force lookup the
kernels carry). With bounce-back these kernels take the interpolated values
as per-row patch lists; rows holding more links than a list takes (256)
put the rest into their ghost slots."""
import numpy as np
import pytest

import synth
from oracle.sim import RELEASE, Config as OConfig, Sim as OSim
from tests.helpers import gpu_config, gpu_lattice, rel_l2

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 2e-3}


@pytest.mark.parametrize("store", [0, 1])
@pytest.mark.parametrize("shape", [(512, 5, 4), (1024, 4, 4), (1536, 4, 5)])
def test_plain_rows(shape, store):
    F = (2e-5, 1e-5, -1e-5)
    u0 = synth.random_velocity(shape, 0.05, seed=31)
    r0 = synth.random_density(shape, 0.01, seed=32)
    o = OSim(OConfig(shape=shape, tau=0.6, body_force=F))
    g = gpu_lattice(gpu_config(nx=shape[0], ny=shape[1], nz=shape[2], tau=0.6, body_force=F, store=store))
    o.set_fields(u0, r0)
    g.set_fields(u0, r0)
    o.step(12)
    g.step(12)
    ug, rg = g.get_fields()
    uo, ro = o.fields()
    assert rel_l2(ug, uo) < TOL[store]
    assert rel_l2(rg - 1, ro - 1) < 50 * TOL[store]
    g.close()


@pytest.mark.parametrize("store", [0, 1])
@pytest.mark.parametrize("bc", ["ibb", "ibm"])
def test_spheres_on_512_rows(bc, store):
    shape = (512, 24, 24)
    spec = synth.hit_spectrum(seed=5, u_rms=0.03, kcut=8)
    u0 = synth.hit_field(spec, shape)
    X = np.array([[40.3, 11.7, 12.2], [260.9, 12.4, 11.1], [505.6, 12.0, 12.8]])  # the last wraps in x
    r = np.full(3, 6.0)
    o = OSim(OConfig(shape=shape, tau=0.55, bc=bc, ibm_retraction=0.4))
    g = gpu_lattice(gpu_config(nx=512, ny=24, nz=24, tau=0.55, bc=1 if bc == "ibb" else 2, ibm_retraction=0.4,
                               store=store, max_particles=3, max_radius=6.0))
    o.set_fields(u0)
    g.set_fields(u0)
    o.set_particles(X, r=r, rho_p=np.full(3, 8.0), mode=RELEASE)
    g.set_particles(X, r, rho_p=8.0, mode=1)
    o.step(10)
    g.step(10)
    ug, _ = g.get_fields()
    uo, _ = o.fields()
    fluid = o.fluid_mask()
    assert rel_l2(ug, uo, fluid) < TOL[store]
    Fg, _, _ = g.forces()
    Fo, _, _ = o.forces()
    assert rel_l2(Fg, Fo) < (1e-4 if store == 0 else 2e-2)
    g.close()


@pytest.mark.parametrize("store", [0, 1])
def test_bounce_back_row_beyond_its_patch_list(store):
    """24 spheres on one line along x: the rows through them hold more links
    than a row's patch list (256), so the link pass puts the rest into their
    ghost slots; fields and forces still match the oracle."""
    shape = (512, 24, 24)
    spec = synth.hit_spectrum(seed=9, u_rms=0.03, kcut=6)
    u0 = synth.hit_field(spec, shape)
    n = 24
    X = np.stack([np.arange(n) * (512.0 / n) + 10.3, np.full(n, 12.2), np.full(n, 11.9)], 1)
    r = np.full(n, 5.0)
    o = OSim(OConfig(shape=shape, tau=0.55, bc="ibb"))
    g = gpu_lattice(gpu_config(nx=512, ny=24, nz=24, tau=0.55, bc=1, store=store, max_particles=n,
                               max_radius=5.0))
    o.set_fields(u0)
    g.set_fields(u0)
    o.set_particles(X, r=r, rho_p=np.full(n, 8.0), mode=RELEASE)
    g.set_particles(X, r, rho_p=8.0, mode=1)
    L = g.links()
    rows = L["node"][:, 2].astype(np.int64) * 24 + L["node"][:, 1]
    assert np.bincount(rows).max() > 256
    o.step(6)
    g.step(6)
    ug, _ = g.get_fields()
    uo, _ = o.fields()
    assert rel_l2(ug, uo, o.fluid_mask()) < TOL[store]
    Fg, _, _ = g.forces()
    Fo, _, _ = o.forces()
    assert rel_l2(Fg, Fo) < (1e-4 if store == 0 else 2e-2)
    g.close()
