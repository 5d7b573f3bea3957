"""Parity of the HIP statistics (lbm_stats) with the FP64 oracle.

Exact-input cases hand the oracle the GPU's own field and particle state, so
the only difference left is FP64 summation order (scalars to 1e-10) and the
bin counts must agree exactly. Full-path cases compare with an oracle run
at the field tolerances of the storage format."""
import numpy as np
import pytest

import synth
from oracle import stats as ostats
from oracle.sim import RELEASE, Config as OConfig, Sim as OSim
from paper_1906_05448_amd import lbm
from tests.helpers import gpu_config, gpu_lattice

pytestmark = pytest.mark.gpu

SCALARS = ["mass", "ke_raw", "ke_masked", "ke_fluid", "eps_raw", "eps_masked", "eps_fluid", "umax", "bulk_u",
           "particle_ke", "particle_ke_rot"]


def _oracle_on_gpu_state(g, cfg, nbins, width, pipe=None):
    u, rho = g.get_fields()
    X, U, W = g.get_particles()
    n = getattr(g, "n_particles", 0)
    keep = getattr(g, "_particles_keep", None)
    r = keep[1] if n else np.zeros(0)
    rp = (keep[4] if keep[4] is not None else np.ones(n)) if n else np.zeros(0)
    nu = (cfg.tau - 0.5) / 3
    return ostats.statistics(u.astype(np.float64), rho.astype(np.float64), nu, cfg.shape, X, U, W, r, rp,
                             pipe=pipe, width=width, nbins=nbins)


def _compare(gs, os_, rtol, count_exact=True, count_rtol=0.0):
    assert gs["n_nodes"] == os_["n_nodes"]
    if count_exact:
        assert gs["n_fluid"] == os_["n_fluid"]
    # sums that cancel (momentum, bulk velocity) are held to the size of
    # their terms: |rho u| <= umax (rho ~ 1) per fluid node
    umax = os_["umax"]
    for k in SCALARS:
        a, b = gs[k], os_[k]
        floor = 1.1 * umax if k == "bulk_u" else 0.0
        assert abs(a - b) <= rtol * (abs(b) + floor) + 1e-300, (k, a, b)
    assert np.allclose(gs["momentum"], os_["momentum"], rtol=0, atol=rtol * 1.1 * umax * os_["n_fluid"])
    hg, ho = gs["hist"], os_["hist"]
    if count_exact:
        assert np.array_equal(hg[0], ho[0])
    else:
        assert np.abs(hg[0] - ho[0]).sum() <= count_rtol * ho[0].sum()
    for k in range(1, 5):
        if ho.shape[1] == 0:
            break
        scale = np.abs(ho[k]).max() + 1e-300
        assert np.abs(hg[k] - ho[k]).max() <= rtol * scale * (1 if count_exact else 50), k


@pytest.mark.parametrize("store", [0, 1])
def test_stats_exact_input_turbulence_no_particles(store):
    shape = (40, 36, 44)
    spec = synth.hit_spectrum(seed=5, u_rms=0.03, kcut=10)
    cfg = gpu_config(nx=shape[0], ny=shape[1], nz=shape[2], tau=0.52, store=store)
    g = gpu_lattice(cfg)
    g.set_fields(synth.hit_field(spec, shape))
    g.step(3)
    gs = g.stats(nbins=0)
    os_ = _oracle_on_gpu_state(g, cfg, 0, 0.25)
    _compare(gs, os_, 1e-10)
    assert gs["eps_raw"] == gs["eps_masked"] and gs["n_fluid"] == gs["n_nodes"]
    g.close()


def test_stats_exact_input_moving_spheres_ibm():
    """Spheres with translation and spin (immersed boundary: the raw field
    inside is the evolving interior fluid), several of them close enough
    that a node is binned by the nearer surface, one across the periodic
    boundary."""
    shape = (48, 40, 44)
    spec = synth.hit_spectrum(seed=6, u_rms=0.03, kcut=10)
    X = np.array([[12.0, 12.5, 13.0], [25.3, 12.9, 13.2], [40.0, 30.0, 30.0], [46.0, 2.0, 42.5]])
    r = np.array([5.0, 5.0, 5.0, 5.0])
    U = np.array([[0.01, 0.0, -0.005], [0.0, 0.02, 0.0], [-0.01, 0.01, 0.01], [0.004, -0.002, 0.003]])
    W = np.array([[0.001, 0.0, 0.0], [0.0, 0.0, -0.002], [0.0005, 0.001, 0.0], [0.0, 0.0015, 0.0]])
    rp = np.array([8.0, 8.0, 6.0, 4.0])
    cfg = gpu_config(nx=shape[0], ny=shape[1], nz=shape[2], tau=0.55, bc=lbm.BC_IBM, ibm_retraction=0.4,
                     max_particles=4, max_radius=5.0)
    g = gpu_lattice(cfg)
    g.set_fields(synth.hit_field(spec, shape))
    g.set_particles(X, r, u=U, omega=W, rho_p=rp, motion=lbm.MOTION_PRESCRIBED)
    for nsteps, nbins in ((0, 32), (4, 40), (3, 64)):
        g.step(nsteps)
        gs = g.stats(nbins=nbins)
        os_ = _oracle_on_gpu_state(g, cfg, nbins, 0.25)
        _compare(gs, os_, 1e-10)
        assert gs["hist"][0].sum() > 1000
    # other bin widths and the multi-slot histogram path
    for nbins, width in ((100, 0.1), (200, 0.07)):
        gs = g.stats(nbins=nbins, bin_width=width)
        os_ = _oracle_on_gpu_state(g, cfg, nbins, width)
        _compare(gs, os_, 1e-10)
    g.close()


def test_stats_exact_input_pipe_wall_ibb():
    shape = (36, 36, 24)
    R, cx, cy = 15.0, 17.5, 17.5
    cfg = gpu_config(nx=shape[0], ny=shape[1], nz=shape[2], tau=0.6, bc=lbm.BC_IBB, wall=lbm.WALL_PIPE_Z,
                     pipe_radius=R, pipe_cx=cx, pipe_cy=cy, body_force=(0.0, 0.0, 2e-6), ibb_max_order=1)
    g = gpu_lattice(cfg)
    g.set_fields(synth.pipe_initial_velocity(shape, R, (cx, cy), 0.03, 0.05, seed=1))
    g.step(20)
    gs = g.stats(nbins=64)
    os_ = _oracle_on_gpu_state(g, cfg, 64, 0.25, pipe=(R, cx, cy))
    _compare(gs, os_, 1e-10)
    assert gs["n_fluid"] < gs["n_nodes"] and gs["bulk_u"] > 0
    g.close()


@pytest.mark.parametrize("store", [0, 1])
def test_stats_full_path_released_spheres_ibb(store):
    """GPU run against an oracle run of the same released spheres
    (bounce-back): masked statistics to the field tolerance."""
    shape = (40, 40, 40)
    spec = synth.hit_spectrum(seed=7, u_rms=0.03, kcut=10)
    u0 = synth.hit_field(spec, shape)
    X = np.array([[10.0, 11.0, 12.0], [29.0, 28.5, 27.0], [10.0, 30.0, 30.0]])
    r = np.full(3, 6.0)
    rp = np.full(3, 4.0)
    o = OSim(OConfig(shape=shape, tau=0.55, bc="ibb"))
    cfg = gpu_config(nx=40, ny=40, nz=40, tau=0.55, bc=lbm.BC_IBB, store=store, max_particles=3, max_radius=6.0)
    g = gpu_lattice(cfg)
    o.set_fields(u0)
    g.set_fields(u0)
    o.set_particles(X, r=r, rho_p=rp, mode=RELEASE)
    g.set_particles(X, r, rho_p=rp, mode=lbm.RELEASE)
    o.step(10)
    g.step(10)
    uo, ro = o.fields()
    P = o.state.P
    os_ = ostats.statistics(uo, ro, (0.55 - 0.5) / 3, shape, P.X, P.U, P.Om, P.r, P.rho, nbins=32)
    gs = g.stats(nbins=32)
    tol = 1e-5 if store == 0 else 2e-3
    for k in ("ke_masked", "ke_fluid", "eps_masked", "eps_fluid", "mass", "umax"):
        assert abs(gs[k] - os_[k]) <= tol * abs(os_[k]), (k, gs[k], os_[k])
    # particle velocities carry the force error (1e-4 FP32, 1e-2 FP16 relative)
    assert abs(gs["particle_ke"] - os_["particle_ke"]) <= (2e-4 if store == 0 else 3e-2) * os_["particle_ke"]
    assert gs["n_fluid"] == os_["n_fluid"]
    assert np.array_equal(gs["hist"][0], os_["hist"][0])
    g.close()


def test_stats_argument_errors_and_empty_histogram():
    g = gpu_lattice(gpu_config(nx=16, ny=16, nz=16))
    for nb, w in ((-1, 0.25), (lbm.STATS_MAX_BINS + 1, 0.25), (8, 0.0), (8, -1.0)):
        with pytest.raises(lbm.LbmError):
            g.stats(nbins=nb, bin_width=w)
    s = g.stats(nbins=0)
    assert s["hist"].shape == (6, 0) and s["n_fluid"] == 16 ** 3
    assert s["ke_raw"] == 0.0 and s["eps_raw"] == 0.0 and abs(s["mass"] - 16 ** 3) < 1e-9
    s = g.stats(nbins=lbm.STATS_MAX_BINS)
    assert s["hist"][0].sum() == 0  # no surface: nothing binned
    g.close()
