"""Pins of the oracle on walls and immersed boundaries against closed forms:
laminar Hagen-Poiseuille pipe flow u_z = g (R^2 - r^2) / (4 nu) reached by
interpolated bounce-back at second order and by the immersed boundary at
first order (Sec. 2.2.1 states IBM is first-order accurate), and the exact
momentum budget of the immersed-boundary step."""
import numpy as np
import pytest

from oracle import collide as col
from oracle.sim import Config, Sim


def _pipe_error(bc, R, rd=0.0):
    n = int(2 * R + 6)
    tau = 1.0
    nu = (tau - 0.5) / 3
    g = 1e-5
    c = (n - 1) / 2
    sim = Sim(Config(shape=(n, n, 4), tau=tau, body_force=(0, 0, g), bc=bc, wall="pipe_z", pipe_radius=R,
                     pipe_cx=c, pipe_cy=c, ibb_max_order=1, ibm_retraction=rd))
    sim.step(int(8 * R * R / nu / 5.78) + 50)          # ~8 slowest decay times
    u = sim.state.u[2, 0]
    x = np.arange(n) - c
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    inside = r2 < R * R
    exact = g * (R * R - r2) / (4 * nu)
    return np.linalg.norm((u - exact)[inside]) / np.linalg.norm(exact[inside])


@pytest.mark.slow
def test_pipe_poiseuille_ibb_second_order():
    e4, e16 = _pipe_error("ibb", 4.0), _pipe_error("ibb", 16.0)
    assert np.log(e4 / e16) / np.log(4.0) > 1.6
    assert e16 < 1e-3


@pytest.mark.slow
def test_pipe_poiseuille_ibm_first_order_and_less_accurate():
    e4, e8 = _pipe_error("ibm", 4.0), _pipe_error("ibm", 8.0)
    order = np.log2(e4 / e8)
    assert 0.5 < order < 1.4
    assert e8 > 5 * _pipe_error("ibb", 8.0)


def test_ibm_step_momentum_budget():
    # The fluid gains N g plus the total spread force, which equals the sum
    # of the marker forces (sum of the delta weights is one); the particle
    # force is minus that sum plus the change of the Kempe inner momentum.
    shape = (18, 16, 17)
    g = np.array([1e-5, 2e-6, -3e-6])
    sim = Sim(Config(shape=shape, tau=0.7, body_force=tuple(g), bc="ibm"))
    from synth import random_velocity
    sim.set_fields(random_velocity(shape, 0.02, seed=9))
    sim.set_particles([[8.3, 7.7, 8.9]], U=[[0.01, 0.0, -0.005]], Om=[[0.0, 0.002, 0.0]], r=[4.2],
                      motion="prescribed")
    N = np.prod(shape)
    for _ in range(3):
        p0 = col.momentum(sim.state.ft).reshape(3, -1).sum(1)
        Iu0 = sim.state.Iu.copy()
        sim.step(1)
        p1 = col.momentum(sim.state.ft).reshape(3, -1).sum(1)
        F, _, _ = sim.forces()
        kempe = sim.state.Iu - Iu0
        assert np.allclose(p1 - p0, N * g - (F[0] - kempe[0]), rtol=0, atol=1e-11)
