"""Pins of the oracle's D3Q19 MRT + Guo core against facts fixed outside it:
published moment-basis norms and equilibrium forms (d'Humieres 2002), the
Guo forcing moment constraints, exact conservation, the BGK limit written
independently here, and hydrodynamic transport coefficients (shear and bulk
viscosity) measured from decaying waves."""
import numpy as np
import pytest

from oracle import collide as col
from oracle.lattice import C, CF, M, OPP, Q, W, relaxation_vector, viscosity
from oracle.sim import Config, Sim


def test_lattice_basics():
    assert Q == 19
    assert abs(W.sum() - 1.0) < 1e-15
    # isotropy: sum w c_a c_b = delta_ab / 3, odd moments vanish
    assert np.allclose(np.einsum("i,ia,ib->ab", W, CF, CF), np.eye(3) / 3, atol=1e-15)
    assert np.allclose(np.einsum("i,ia->a", W, CF), 0, atol=1e-15)
    assert (C[OPP] == -C).all()


def test_moment_basis_published_norms():
    # d'Humieres et al. 2002 list the squared norms of the D3Q19 basis rows.
    norms = [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8]
    G = M @ M.T
    assert np.allclose(G, np.diag(norms), atol=1e-12)


def test_equilibrium_moments_match_dhumieres_forms():
    # d'Humieres 2002 equilibria with omega_eps = 3, omega_epsj = -11/2,
    # omega_xx = -1/2 (the values that reproduce the second-order
    # polynomial equilibrium).
    rng = np.random.default_rng(3)
    for _ in range(5):
        rho = 1.0 + 0.05 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(3)
        j = rho * u
        jj = j @ j
        meq = M @ col.equilibrium(rho, u.reshape(3))
        exp = [rho, -11 * rho + 19 * jj / rho, 3 * rho - 5.5 * jj / rho,
               j[0], -2 / 3 * j[0], j[1], -2 / 3 * j[1], j[2], -2 / 3 * j[2],
               (3 * j[0] ** 2 - jj) / rho, -0.5 * (3 * j[0] ** 2 - jj) / rho,
               (j[1] ** 2 - j[2] ** 2) / rho, -0.5 * (j[1] ** 2 - j[2] ** 2) / rho,
               j[0] * j[1] / rho, j[1] * j[2] / rho, j[0] * j[2] / rho, 0, 0, 0]
        assert np.allclose(meq, exp, atol=1e-14)


def test_guo_source_moment_constraints():
    # Guo, Zheng & Shi 2002: sum F_i = 0, sum c F_i = F, sum c c F_i = uF + Fu.
    rng = np.random.default_rng(4)
    u = 0.05 * rng.standard_normal(3)
    F = 1e-3 * rng.standard_normal(3)
    Fb = col.guo_source(u, F)
    assert abs(Fb.sum()) < 1e-17
    assert np.allclose(CF.T @ Fb, F, atol=1e-17)
    assert np.allclose(np.einsum("i,ia,ib->ab", Fb, CF, CF), np.outer(u, F) + np.outer(F, u), atol=1e-17)


def test_conservation_periodic_box():
    # Mass is conserved exactly; momentum grows by N*F per step.
    shape = (12, 10, 8)
    F = np.array([1e-5, -2e-5, 3e-6])
    cfg = Config(shape=shape, tau=0.7, body_force=tuple(F))
    sim = Sim(cfg)
    rng = np.random.default_rng(5)
    sim.state.ft = col.equilibrium(np.ones(cfg.zyx), np.zeros((3,) + cfg.zyx)) * \
        (1 + 0.02 * rng.standard_normal((Q,) + cfg.zyx))
    m0 = sim.state.ft.sum()
    p0 = col.momentum(sim.state.ft).reshape(3, -1).sum(1)
    nsteps = 25
    sim.step(nsteps)
    N = np.prod(shape)
    assert abs(sim.state.ft.sum() - m0) / m0 < 1e-13
    p = col.momentum(sim.state.ft).reshape(3, -1).sum(1)
    assert np.allclose(p, p0 + nsteps * N * F, rtol=0, atol=1e-12 * m0)


def _bgk_step(ft, tau, F):
    """Single-relaxation BGK with Guo forcing, written out here in population
    space: f~ = f - (f - feq)/tau + (1 - 1/(2 tau)) Fbar."""
    f = np.empty_like(ft)
    for i in range(19):
        f[i] = np.roll(ft[i], shift=(C[i, 2], C[i, 1], C[i, 0]), axis=(0, 1, 2))
    rho = f.sum(0)
    mom = np.einsum("ia,i...->a...", CF, f)
    u = (mom + 0.5 * F[:, None, None, None]) / rho
    out = np.empty_like(f)
    for i in range(19):
        cu = CF[i, 0] * u[0] + CF[i, 1] * u[1] + CF[i, 2] * u[2]
        uu = (u * u).sum(0)
        feq = W[i] * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * uu)
        cF = CF[i] @ F
        uF = F[0] * u[0] + F[1] * u[1] + F[2] * u[2]
        src = W[i] * (3 * (cF - uF) + 9 * cu * cF)
        out[i] = f[i] - (f[i] - feq) / tau + (1 - 0.5 / tau) * src
    return out


def test_mrt_with_equal_rates_is_bgk():
    tau = 0.83
    shape = (6, 5, 7)
    F = np.array([2e-5, 1e-5, -1e-5])
    cfg = Config(shape=shape, tau=tau, s_e=1 / tau, s_eps=1 / tau, s_q=1 / tau, s_pi=1 / tau, s_m=1 / tau,
                 body_force=tuple(F))
    sim = Sim(cfg)
    rng = np.random.default_rng(6)
    sim.set_fields(0.05 * rng.standard_normal((3,) + cfg.zyx), 1 + 0.01 * rng.standard_normal(cfg.zyx))
    ft = sim.state.ft.copy()
    for _ in range(4):
        sim.step(1)
        ft = _bgk_step(ft, tau, F)
    assert np.abs(sim.state.ft - ft).max() < 1e-14


def _decay_rate(amplitudes, steps):
    t = np.arange(len(amplitudes)) * steps
    return -np.polyfit(t, np.log(amplitudes), 1)[0]


@pytest.mark.parametrize("diagonal", [False, True])
def test_shear_wave_viscosity(diagonal):
    # A shear wave decays as exp(-nu k^2 t); nu = (tau - 1/2)/3 for the stress
    # moments (both the off-diagonal p_xy and the diagonal p_xx - p_yy pair).
    tau = 0.8
    N = 32
    A = 1e-4
    if diagonal:
        shape = (N, N, 4)
        cfg = Config(shape=shape, tau=tau)
        z, y, x = np.meshgrid(np.arange(4), np.arange(N), np.arange(N), indexing="ij")
        ph = 2 * np.pi * (x + y) / N
        u = np.stack([A * np.sin(ph), -A * np.sin(ph), 0 * ph])
        k2 = 2 * (2 * np.pi / N) ** 2
        def amp(uu):
            return np.sqrt(((uu[0] * np.sin(ph)).mean() * 2) ** 2)
    else:
        shape = (4, N, 4)
        cfg = Config(shape=shape, tau=tau)
        z, y, x = np.meshgrid(np.arange(4), np.arange(N), np.arange(4), indexing="ij")
        ph = 2 * np.pi * y / N
        u = np.stack([A * np.sin(ph), 0 * ph, 0 * ph])
        k2 = (2 * np.pi / N) ** 2
        def amp(uu):
            return abs((uu[0] * np.sin(ph)).mean() * 2)
    sim = Sim(cfg)
    sim.set_fields(u)
    amps = []
    for _ in range(12):
        sim.step(40)
        amps.append(amp(sim.state.u))
    nu = _decay_rate(np.array(amps), 40) / k2
    assert abs(nu / viscosity(tau) - 1) < 0.01


@pytest.mark.parametrize("s_e", [1.19, 1.6])
def test_sound_wave_bulk_viscosity(s_e):
    # Acoustic energy of a standing wave decays at (4/3 nu + zeta) k^2 with the
    # D3Q19 MRT bulk viscosity zeta = (2/9)(1/s_e - 1/2) (d'Humieres 2002).
    tau = 0.8
    N = 64
    cfg = Config(shape=(N, 4, 4), tau=tau, s_e=s_e)
    z, y, x = np.meshgrid(np.arange(4), np.arange(4), np.arange(N), indexing="ij")
    sim = Sim(cfg)
    sim.set_fields(np.zeros((3,) + cfg.zyx), 1 + 1e-5 * np.cos(2 * np.pi * x / N))
    k2 = (2 * np.pi / N) ** 2
    energies = []
    period = N * np.sqrt(3)          # acoustic period 2 pi / (c_s k)
    times = []
    t = 0
    for _ in range(10):
        sim.step(37)
        t += 37
        rho, u = sim.state.rho, sim.state.u
        e = ((rho - 1) ** 2 / 3 + (rho * u[0]) ** 2).mean()
        energies.append(e)
        times.append(t)
    rate = -np.polyfit(np.array(times), np.log(energies), 1)[0]
    nu = viscosity(tau)
    zeta = 2 / 9 * (1 / s_e - 0.5)
    assert abs(rate / ((4 / 3 * nu + zeta) * k2) - 1) < 0.03, (rate, period)


def test_uniform_equilibrium_is_fixed_point():
    cfg = Config(shape=(5, 4, 6), tau=0.55)
    sim = Sim(cfg)
    u = np.broadcast_to(np.array([0.03, -0.02, 0.01]).reshape(3, 1, 1, 1), (3,) + cfg.zyx)
    sim.set_fields(u, 1.02 * np.ones(cfg.zyx))
    ft0 = sim.state.ft.copy()
    sim.step(3)
    assert np.abs(sim.state.ft - ft0).max() < 1e-15
