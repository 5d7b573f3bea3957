"""Parity of the HIP energy and dissipation spectra (lbm_spectrum) with the
FP64 oracle's spectra (numpy FFT and shell binning).

Every case hands the oracle the GPU's own field and particle state, so what
is compared is the masking, the FP32 transform and the shell sums. The
transform's rounding is about log2(N) FP32 ulps of the field, so each shell
is held to 2e-6 of the total energy; Parseval to 1e-6 of it."""
import numpy as np
import pytest

import synth
from oracle import stats as ostats
from oracle.sim import RELEASE
from paper_1906_05448_amd import lbm
from tests.helpers import gpu_config, gpu_lattice

pytestmark = pytest.mark.gpu


def _largest_shell(shape):
    return int(np.floor(np.sqrt(sum((n // 2) ** 2 for n in shape)) + 0.5))


def _oracle(g, shape, masked, kmax):
    u, _ = g.get_fields()
    u = u.astype(np.float64)
    if masked and getattr(g, "n_particles", 0):
        X, U, W = g.get_particles()
        r = g._particles_keep[1]
        owner, _ = ostats.classify(shape, X, r, None, 0.25, 0)
        u = ostats.masked_velocity(u, owner, X, U, W, shape)
    _, E = ostats.energy_spectrum(u, kmax)
    return u, E


def _check(g, shape, masked, tau):
    kmax = _largest_shell(shape)
    k, E, D = g.spectrum(kmax, masked=masked)
    u, Eo = _oracle(g, shape, masked, kmax)
    total = Eo.sum()
    assert total > 0
    assert np.abs(E - Eo).max() <= 2e-6 * total
    # Parseval on the field the spectrum was taken of
    assert abs(E.sum() - 0.5 * (u * u).sum(0).mean()) <= 1e-6 * total
    nu = (tau - 0.5) / 3
    assert np.array_equal(D, 2.0 * nu * k * k * E)
    # fixed summation order: the same spectrum on a second call
    _, E2, _ = g.spectrum(kmax, masked=masked)
    assert np.array_equal(E, E2)
    # truncation at a smaller kmax reports the same shells
    _, E3, _ = g.spectrum(3, masked=masked)
    assert np.array_equal(E3, E[:4])
    return E


@pytest.mark.parametrize("shape", [(32, 16, 64), (64, 64, 64), (16, 32, 1024), (1024, 16, 32)])
def test_spectrum_turbulence_no_particles(shape):
    spec = synth.hit_spectrum(seed=5, u_rms=0.04, kcut=6)
    u0 = synth.hit_field(spec, shape)
    g = gpu_lattice(gpu_config(nx=shape[0], ny=shape[1], nz=shape[2], tau=0.6, store=0))
    g.set_fields(u0)
    g.step(3)
    E = _check(g, shape, masked=False, tau=0.6)
    # without particles masking changes nothing
    _, Em, _ = g.spectrum(len(E) - 1, masked=True)
    assert np.array_equal(Em, E)
    g.close()


@pytest.mark.parametrize("bc", [1, 2])
def test_spectrum_masked_released_spheres(bc):
    shape = (64, 32, 32)
    spec = synth.hit_spectrum(seed=7, u_rms=0.04, kcut=6)
    u0 = synth.hit_field(spec, shape)
    X = np.array([[12.0, 10.0, 9.0], [40.5, 20.0, 16.0], [62.5, 30.5, 1.0]])
    r = np.full(3, 5.0)
    kw = dict(nx=shape[0], ny=shape[1], nz=shape[2], tau=0.6, store=0, bc=bc, max_particles=3, max_radius=5.0)
    if bc == 2:
        kw["ibm_retraction"] = 0.0
    g = gpu_lattice(gpu_config(**kw))
    g.set_fields(u0)
    # rho_p = 4: the explicit immersed-boundary coupling diverges for
    # neutrally buoyant spheres this small (the oracle does too)
    g.set_particles(X, r, rho_p=np.full(3, 4.0), mode=RELEASE)
    g.step(4)
    Em = _check(g, shape, masked=True, tau=0.6)
    if bc == 2:
        # the immersed boundary keeps a virtual fluid inside: both forms
        Eu = _check(g, shape, masked=False, tau=0.6)
        assert not np.array_equal(Em, Eu)
    g.close()


def test_spectrum_needs_power_of_two_sides():
    g = gpu_lattice(gpu_config(nx=48, ny=32, nz=32, tau=0.6, store=0))
    with pytest.raises(lbm.LbmError):
        g.spectrum(4)
    g.close()
