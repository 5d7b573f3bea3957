"""Overlap mode (lbm_set_overlap) moves the particle stage and the next
step's geometry onto a second stream beside the stream-collide kernel; the
kernels and their inputs are the same, so every result must be bit-identical
to the serial order: bounce-back and immersed boundary, FP32 and FP16, over
steps in which released spheres move, touch and uncover nodes."""
import numpy as np
import pytest

import synth
from paper_1906_05448_amd import lbm
from tests.helpers import gpu_config, gpu_lattice

pytestmark = pytest.mark.gpu

SHAPE = (48, 44, 40)
X = np.array([[10.0, 10.0, 10.0], [20.6, 10.3, 10.0], [30.0, 28.0, 25.0], [12.0, 30.0, 28.0],
              [36.0, 12.0, 30.0], [46.5, 2.0, 38.7]])


def _run(bc, store, overlap):
    g = gpu_lattice(gpu_config(nx=SHAPE[0], ny=SHAPE[1], nz=SHAPE[2], tau=0.55, bc=bc, store=store,
                               ibm_retraction=0.4 if bc == lbm.BC_IBM else 0.0, max_particles=6, max_radius=5.0,
                               coll_restitution=0.9, coll_tc_steps=8.0))
    spec = synth.hit_spectrum(seed=3, u_rms=0.04, kcut=10)
    g.set_fields(synth.hit_field(spec, SHAPE))
    g.set_particles(X, np.full(6, 5.0), rho_p=np.full(6, 8.0), mode=lbm.RELEASE)
    g.set_overlap(overlap)
    out = []
    for _ in range(3):
        g.step(10)
        out.append([*g.get_fields(), *g.get_particles(), *g.forces()])
    out.append(list(g.geometry_counts() if bc == lbm.BC_IBB else g.ibm_support()))
    g.close()
    return out


@pytest.mark.parametrize("bc,store", [(lbm.BC_IBB, lbm.STORE_F32), (lbm.BC_IBB, lbm.STORE_F16S),
                                      (lbm.BC_IBM, lbm.STORE_F32), (lbm.BC_IBM, lbm.STORE_F16S)])
def test_overlap_is_bit_identical(bc, store):
    serial, overlapped = _run(bc, store, False), _run(bc, store, True)
    moved = np.abs(serial[-2][2] - X).max()
    assert moved > 0.05  # the spheres moved by a fraction of a node
    for a, b in zip(serial, overlapped):
        for u, v in zip(a, b):
            assert np.array_equal(np.asarray(u), np.asarray(v), equal_nan=True)
