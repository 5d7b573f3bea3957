"""Parity of the HIP pipe TKE-budget accumulator (lbm_pipe_budget_*) with the
FP64 oracle (Eq. (1a)-(1c)).

The oracle is handed the GPU's own snapshots, so what is compared is the
masking, the cylindrical quantities, the bin sums (FP64, different order:
1e-10 of each moment's scale) and the assembly of the 13 terms (1e-7 of each
term's scale; empty bins NaN on both sides)."""
import numpy as np
import pytest

import synth
from oracle import pipe_budget as opb
from oracle import stats as ostats
from paper_1906_05448_amd import lbm
from tests.helpers import gpu_config, gpu_lattice

pytestmark = pytest.mark.gpu

TAU = 0.56


def _lattice(shape, pipe, bc, lattice=0):
    R, cx, cy = pipe
    kw = dict(nx=shape[0], ny=shape[1], nz=shape[2], tau=TAU, body_force=(0.0, 0.0, 2e-5), bc=bc, wall=1,
              pipe_radius=R, pipe_cx=cx, pipe_cy=cy, store=0, lattice=lattice)
    if bc == 1:
        kw["ibb_max_order"] = 1
    return gpu_lattice(gpu_config(**kw))


def _oracle_add(M, g, shape, pipe, w):
    u, rho = g.get_fields()
    none = np.zeros((0, 3))
    owner, _ = ostats.classify(shape, none, np.zeros(0), pipe, 0.25, 0)
    um = ostats.masked_velocity(u.astype(np.float64), owner, none, none, none, shape)
    opb.add_snapshot(M, um, rho.astype(np.float64), shape, pipe, w)


@pytest.mark.parametrize("bc,lattice", [(1, lbm.LATTICE_D3Q19), (2, lbm.LATTICE_D3Q19), (1, lbm.LATTICE_D3Q27)])
def test_pipe_budget_matches_oracle(bc, lattice):
    shape = (32, 30, 24)
    pipe = (11.3, 15.4, 14.6)
    w = 0.75
    g = _lattice(shape, pipe, bc, lattice)
    spec = synth.hit_spectrum(seed=11, u_rms=0.01, kcut=5)
    g.set_fields(synth.hit_field(spec, shape))
    g.step(5)
    g.pipe_budget_reset(w)
    nb = int(np.ceil(pipe[0] / w))
    M = np.zeros((len(opb.MOMENTS), nb))
    for _ in range(3):
        g.step(4)
        g.pipe_budget_add()
        _oracle_add(M, g, shape, pipe, w)
    ns, Mg, Tg = g.pipe_budget_read()
    assert ns == 3 and Mg.shape == M.shape
    assert np.array_equal(Mg[0], M[0])  # node counts per bin
    # each moment against its own scale, except the strain and gradient
    # sums (rows 5-19), held to their common scale: sums such as d_z u_r
    # cancel over the periodic z direction down to rounding
    scale = np.abs(M).max(axis=1, keepdims=True)
    scale[5:20] = np.abs(M[5:20]).max()
    assert np.all(np.abs(Mg - M) <= 1e-10 * scale + 1e-300)
    To = opb.budget_terms(M, w, (TAU - 0.5) / 3.0)
    assert np.array_equal(np.isnan(Tg), np.isnan(To))
    ok = ~np.isnan(To)
    # the terms are rates of one balance: held to their common scale
    assert np.all(np.abs(Tg - To)[ok] <= 1e-7 * np.abs(To[ok]).max())
    assert np.abs(To[:, ok.all(0)]).max() > 0
    # a fixed summation order: the same snapshot gives the same sums
    g.pipe_budget_reset(w)
    g.pipe_budget_add()
    _, M1, _ = g.pipe_budget_read()
    g.pipe_budget_reset(w)
    g.pipe_budget_add()
    _, M2, _ = g.pipe_budget_read()
    assert np.array_equal(M1, M2)
    g.close()


def test_pipe_budget_errors():
    g = gpu_lattice(gpu_config(nx=16, ny=16, nz=8, tau=0.6, store=0))
    with pytest.raises(lbm.LbmError):  # no pipe wall
        g.pipe_budget_reset(0.5)
    g.close()
    g = _lattice((24, 24, 8), (9.3, 11.5, 11.7), 1)
    with pytest.raises(lbm.LbmError):  # not reset
        g.pipe_budget_add()
    with pytest.raises(lbm.LbmError):  # more bins than allowed
        g.pipe_budget_reset(1e-3)
    g.pipe_budget_reset(0.5)
    g.pipe_budget_add()
    ns, M, T = g.pipe_budget_read()
    assert ns == 1 and M.shape == (38, 19) and T.shape == (13, 19)
    g.close()
