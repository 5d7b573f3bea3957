"""Parity of the HIP D3Q27 pipe solver (Sec. 2.2: one relaxation parameter,
optional energy-mode rate; linear bounce-back pipe wall) with the FP64
oracle, through the C ABI.

Tolerances: velocity 1e-5 relative L2 (FP32 storage and arithmetic), density
deviation 5e-4 relative L2 (rho - 1 is small, so its relative error carries
the FP32 rounding of rho itself); wall links compared exactly by node,
direction and scheme, q to FP32 rounding."""
import numpy as np
import pytest

import synth
from oracle import d3q27 as q27
from paper_1906_05448_amd import lbm
from tests.helpers import gpu_config, gpu_lattice, rel_l2

pytestmark = pytest.mark.gpu


def _cfg(shape, tau, tau_bulk, F, pipe=None):
    kw = dict(nx=shape[0], ny=shape[1], nz=shape[2], tau=tau, tau_bulk=tau_bulk, body_force=tuple(F),
              lattice=lbm.LATTICE_D3Q27, store=0)
    if pipe is not None:
        kw.update(bc=lbm.BC_IBB, wall=lbm.WALL_PIPE_Z, ibb_max_order=1, pipe_radius=pipe[0], pipe_cx=pipe[1],
                  pipe_cy=pipe[2])
    return gpu_config(**kw)


def _pair(shape, tau, tau_bulk, F, u0, r0, steps, pipe=None):
    o = q27.Sim27(shape, tau, tau_bulk, F, pipe)
    o.set_fields(u0, r0)
    o.step(steps)
    g = gpu_lattice(_cfg(shape, tau, tau_bulk, F, pipe))
    g.set_fields(u0, r0)
    g.step(steps)
    ug, rg = g.get_fields()
    return g, ug, rg, o


@pytest.mark.parametrize("tau_bulk,shape", [(0.0, (150, 13, 9)), (1.3, (150, 13, 9)), (1.3, (256, 7, 5))])
def test_periodic_ragged_tiles(tau_bulk, shape):
    # 150 x 13 x 9: 64 x 4 tiles (they fill a 150-node row better than
    # 128 x 2), a ragged x tail, a ragged y tail; 256 x 7 x 5: 128 x 2 tiles
    # with an odd y
    F = (1e-5, -2e-5, 3e-5)
    u0 = synth.random_velocity(shape, 0.05, seed=21)
    r0 = synth.random_density(shape, 0.01, seed=22)
    g, ug, rg, o = _pair(shape, 0.58, tau_bulk, F, u0, r0, 20)
    g.close()
    assert rel_l2(ug, o.u) < 1e-5
    assert rel_l2(rg - 1, o.rho - 1) < 5e-4


def test_minimum_box_and_zero_steps():
    shape = (4, 4, 4)
    u0 = synth.random_velocity(shape, 0.03, seed=3)
    g = gpu_lattice(_cfg(shape, 0.9, 2.0, (1e-4, 0, 0)))
    g.set_fields(u0)
    ug, _ = g.get_fields()
    assert np.allclose(ug, u0, rtol=0, atol=1e-7)
    g.close()
    g, ug, rg, o = _pair(shape, 0.9, 2.0, (1e-4, 0, 0), u0, None, 10)
    g.close()
    assert rel_l2(ug, o.u) < 1e-5


@pytest.mark.parametrize("tau_bulk", [0.0, 0.9])
def test_pipe_wall_matches_oracle(tau_bulk):
    shape = (32, 30, 12)
    pipe = (11.3, 15.4, 14.6)
    F = (0.0, 0.0, 2e-5)
    u0 = synth.pipe_initial_velocity(shape, pipe[0], pipe[1:], 0.03, 0.1, seed=5)
    g, ug, rg, o = _pair(shape, 0.56, tau_bulk, F, u0, None, 30, pipe)
    fluid = ~o.solid
    assert rel_l2(ug[:, fluid], o.u[:, fluid]) < 1e-5
    assert rel_l2(rg[fluid] - 1, o.rho[fluid] - 1) < 5e-4
    # the wall links: same set, same schemes, q to FP32 rounding
    L = g.links()
    g.close()
    OL = o.links
    key_g = {(tuple(n), tuple(d)): (q, s) for n, d, q, s in zip(L["node"], L["dir"], L["q"], L["scheme"])}
    key_o = {(tuple(n), tuple(q27.C[a])): (q, s) for n, a, q, s in zip(OL["xf"], OL["a"], OL["q"], OL["scheme"])}
    assert len(key_g) == len(L["q"]) and set(key_g) == set(key_o)
    assert (L["particle"] == -1).all()
    for k, (q, s) in key_g.items():
        qo, so = key_o[k]
        assert s == so
        assert abs(q - qo) <= 1e-6 * max(qo, 1e-3)


def test_full_pipe_z_periodic_translation():
    """The 160 x 160 x 480 pipe of the measured workload, started from a field
    of z period 12: its state after three steps is the 160 x 160 x 12 pipe's
    at every node (translation invariance along the axis), which the oracle
    computes in full."""
    R, c = 74.5, (79.5, 79.5)
    small, full = (160, 160, 12), (160, 160, 480)
    u_s = synth.pipe_initial_velocity(small, R, c, 0.05, 0.1, seed=9)
    o = q27.Sim27(small, 0.52, 0.0, (0, 0, 7e-6), (R, c[0], c[1]))
    o.set_fields(u_s)
    o.step(3)
    g = gpu_lattice(_cfg(full, 0.52, 0.0, (0, 0, 7e-6), (R, c[0], c[1])))
    g.set_fields(np.tile(u_s, (1, full[2] // small[2], 1, 1)))
    g.step(3)
    ug, rg = g.get_fields()
    g.close()
    fluid = ~o.solid
    for k in range(0, full[2], small[2]):
        blk = ug[:, k:k + small[2]]
        assert rel_l2(blk[:, fluid], o.u[:, fluid]) < 1e-5, k
    assert rel_l2(rg[:12][fluid] - 1, o.rho[fluid] - 1) < 5e-4


def test_configuration_errors():
    base = dict(nx=16, ny=16, nz=8, lattice=lbm.LATTICE_D3Q27)
    for bad in (dict(store=1), dict(bc=lbm.BC_IBM), dict(tau_bulk=0.4),
                dict(bc=lbm.BC_IBB, max_particles=4, max_radius=2.0),
                dict(bc=lbm.BC_IBB, wall=lbm.WALL_PIPE_Z, pipe_radius=6.0, pipe_cx=7.5, pipe_cy=7.5, ibb_max_order=2)):
        with pytest.raises(lbm.LbmError):
            gpu_lattice(gpu_config(**base, **bad))
    with pytest.raises(lbm.LbmError):  # the knob belongs to the D3Q27 solver
        gpu_lattice(gpu_config(nx=16, ny=16, nz=8, tau_bulk=1.0))


def test_instability_is_reported():
    g = gpu_lattice(_cfg((8, 8, 8), 0.6, 0.0, (0, 0, 0)))
    u = np.zeros((3, 8, 8, 8))
    u[0] = 0.4                      # above the |u| < 0.35 guard
    g.set_fields(u)
    g.step(1)
    with pytest.raises(lbm.LbmError) as ei:
        g.sync()
    assert ei.value.status == -5
    g.sync()                        # the latch clears once reported
    g.close()
