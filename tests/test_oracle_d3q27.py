"""Pins of the FP64 D3Q27 oracle (the pipe solver of Sec. 2.2) against what
the lattice and the hydrodynamics fix: the weights' isotropy tensors, an
orthogonal moment basis, the reduction of the single-parameter collision to
BGK, exact conservation, the separate relaxation of the traceless and trace
parts of the stress, the shear-wave decay rate nu k^2, the sound attenuation
(k^2/2)(4 nu/3 + 2 nu_b/3) with and without the bulk-viscosity knob, and
second-order Hagen-Poiseuille flow with the linear bounce-back wall."""
import numpy as np
import pytest

from oracle import d3q27 as q27

D = np.eye(3)


def test_weights_isotropy():
    c, w = q27.CF, q27.W
    assert q27.Q == 27 and np.isclose(w.sum(), 1.0, rtol=0, atol=1e-15)
    assert np.allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), D / 3, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0, atol=1e-16)
    iso4 = (np.einsum("ab,cd->abcd", D, D) + np.einsum("ac,bd->abcd", D, D) + np.einsum("ad,bc->abcd", D, D)) / 9
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso4, atol=1e-16)
    assert sorted(set(np.round(w * 216).astype(int))) == [1, 4, 16, 64]
    assert (q27.C[q27.OPP] == -q27.C).all()


def test_basis_orthogonal_and_energy_row():
    G = q27.M @ np.diag(q27.W) @ q27.M.T
    assert np.allclose(G - np.diag(np.diag(G)), 0, atol=1e-14)
    assert np.allclose(q27.M[q27.ROW_E], (q27.CF ** 2).sum(1) - 1.0)
    assert np.allclose(q27.M[q27.ROW_RHO], 1.0)
    for k, r in enumerate(q27.ROWS_J):
        assert np.array_equal(q27.M[r], q27.CF[:, k])


def _random_state(rng, n=50):
    rho = 1.0 + 0.05 * rng.standard_normal(n)
    u = 0.05 * rng.standard_normal((3, n))
    f = q27.equilibrium(rho, u) * (1.0 + 0.05 * rng.standard_normal((27, n)))
    F = 1e-3 * rng.standard_normal((3, n))
    return f, F


def test_equilibrium_and_source_moments():
    rng = np.random.default_rng(1)
    rho = 1.0 + 0.1 * rng.random(8)
    u = 0.1 * rng.standard_normal((3, 8))
    F = rng.standard_normal((3, 8))
    c = q27.CF
    feq = q27.equilibrium(rho, u)
    assert np.allclose(feq.sum(0), rho, rtol=1e-14)
    assert np.allclose(np.einsum("ia,in->an", c, feq), rho * u, atol=1e-15)
    P = np.einsum("ia,ib,in->abn", c, c, feq)
    assert np.allclose(P, rho * (np.einsum("an,bn->abn", u, u) + D[:, :, None] / 3), atol=1e-15)
    S = q27.guo_source(u, F)
    assert np.allclose(S.sum(0), 0, atol=1e-14)
    assert np.allclose(np.einsum("ia,in->an", c, S), F, atol=1e-14)
    assert np.allclose(np.einsum("ia,ib,in->abn", c, c, S),
                       np.einsum("an,bn->abn", u, F) + np.einsum("an,bn->abn", F, u), atol=1e-14)


def test_single_parameter_is_bgk():
    """tau_bulk = tau: the moment-space collision equals BGK with Guo forcing
    written in population space."""
    rng = np.random.default_rng(2)
    f, F = _random_state(rng)
    tau = 0.63
    ft, rho, u = q27.collide(f, F, q27.relaxation_vector(tau))
    bgk = f - (f - q27.equilibrium(rho, u)) / tau + (1 - 0.5 / tau) * q27.guo_source(u, F)
    assert np.allclose(ft, bgk, rtol=0, atol=1e-15)
    assert np.allclose(u, (np.einsum("ia,in->an", q27.CF, f) + 0.5 * F) / f.sum(0), atol=1e-16)


@pytest.mark.parametrize("tau_bulk", [0.0, 0.9, 2.5])
def test_conservation(tau_bulk):
    rng = np.random.default_rng(3)
    f, F = _random_state(rng)
    ft, _, _ = q27.collide(f, F, q27.relaxation_vector(0.7, tau_bulk))
    assert np.allclose(ft.sum(0), f.sum(0), rtol=1e-15, atol=0)
    j0 = np.einsum("ia,in->an", q27.CF, f)
    j1 = np.einsum("ia,in->an", q27.CF, ft)
    assert np.allclose(j1 - j0, F, rtol=0, atol=1e-15)


def test_stress_relaxation_traceless_and_trace():
    """F = 0: the non-equilibrium stress keeps its traceless part times
    (1 - 1/tau) and its trace times (1 - 1/tau_bulk)."""
    rng = np.random.default_rng(4)
    f, _ = _random_state(rng)
    F = np.zeros((3, f.shape[1]))
    tau, tb = 0.7, 1.9
    ft, rho, u = q27.collide(f, F, q27.relaxation_vector(tau, tb))
    feq = q27.equilibrium(rho, u)
    c = q27.CF
    P0 = np.einsum("ia,ib,in->abn", c, c, f - feq)
    P1 = np.einsum("ia,ib,in->abn", c, c, ft - feq)
    tr0, tr1 = np.einsum("aan->n", P0), np.einsum("aan->n", P1)
    dev0 = P0 - D[:, :, None] * tr0 / 3
    dev1 = P1 - D[:, :, None] * tr1 / 3
    assert np.allclose(tr1, (1 - 1 / tb) * tr0, atol=1e-15)
    assert np.allclose(dev1, (1 - 1 / tau) * dev0, atol=1e-15)
    assert np.abs(tr0).max() > 1e-4 and np.abs(dev0).max() > 1e-4


def _shear_amp(sim, L):
    y = np.arange(L)
    return 2.0 / L * (sim.u[0, 0, :, 0] * np.sin(2 * np.pi * y / L)).sum()


@pytest.mark.parametrize("tau_bulk", [0.0, 2.0])
def test_shear_wave_decay(tau_bulk):
    L, tau, U = 32, 0.8, 1e-4
    nu = (tau - 0.5) / 3
    sim = q27.Sim27((4, L, 4), tau, tau_bulk)
    y = np.arange(L)
    u = np.zeros((3, 4, L, 4))
    u[0] = U * np.sin(2 * np.pi * y / L)[None, :, None]
    sim.set_fields(u)
    sim.step(50)
    a0 = _shear_amp(sim, L)
    sim.step(250)
    a1 = _shear_amp(sim, L)
    nu_fit = np.log(a0 / a1) / (250 * (2 * np.pi / L) ** 2)
    assert abs(nu_fit / nu - 1) < 5e-3


@pytest.mark.parametrize("tau_bulk", [0.0, 2.0])
def test_sound_attenuation(tau_bulk):
    """Standing wave rho' = e cos(kx): the acoustic energy c_s^2 a^2 + b^2
    decays as exp(-2 Gamma t), Gamma = (k^2/2)(4 nu/3 + 2 nu_b/3)."""
    L, tau, e = 64, 0.8, 1e-5
    nu = (tau - 0.5) / 3
    nub = ((tau if tau_bulk == 0.0 else tau_bulk) - 0.5) / 3
    k = 2 * np.pi / L
    x = np.arange(L)
    sim = q27.Sim27((L, 2, 2), tau, tau_bulk)
    sim.set_fields(np.zeros((3, 2, 2, L)), 1.0 + e * np.cos(k * x)[None, None, :] * np.ones((2, 2, L)))
    t, E = [], []
    for n in range(1, 1201):
        sim.step()
        if n >= 100:
            a = 2.0 / L * ((sim.rho[0, 0] - 1.0) * np.cos(k * x)).sum()
            b = 2.0 / L * (sim.u[0, 0, 0] * np.sin(k * x)).sum()
            t.append(n)
            E.append(a * a / 3.0 + b * b)
    slope = np.polyfit(np.array(t), np.log(np.array(E)), 1)[0]
    gamma = (k * k / 2) * (4 * nu / 3 + 2 * nub / 3)
    assert abs(-slope / 2 / gamma - 1) < 0.03


def _pipe_error(R):
    n = int(2 * R + 6)
    tau, g = 1.0, 1e-5
    nu = (tau - 0.5) / 3
    c = (n - 1) / 2
    sim = q27.Sim27((n, n, 2), tau, 0.0, (0, 0, g), pipe=(R, c, c))
    sim.step(int(8 * R * R / nu / 5.78) + 50)
    u = sim.u[2, 0]
    x = np.arange(n) - c
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    inside = r2 < R * R
    exact = g * (R * R - r2) / (4 * nu)
    assert np.isfinite(u[inside]).all()
    return np.linalg.norm((u - exact)[inside]) / np.linalg.norm(exact[inside])


@pytest.mark.slow
def test_pipe_poiseuille_linear_bounce_back_second_order():
    # steady (16 decay times give the same errors): 2.4e-2 and 1.6e-3
    e4, e16 = _pipe_error(4.0), _pipe_error(16.0)
    assert np.log(e4 / e16) / np.log(4.0) > 1.6
    assert e16 < 3e-3


def test_pipe_links_cover_every_wall_neighbour():
    """Every pull from a solid node into a fluid node is a link (the NaN
    interior would otherwise reach the fluid), and q is in [0, 1)."""
    links, solid = q27.pipe_links((20, 18, 3), 7.3, 9.6, 8.2)
    assert len(links["a"]) > 0
    assert (links["q"] >= 0).all() and (links["q"] < 1).all()
    cz = q27.C[links["a"], 2]
    assert (cz != 0).any() and (cz == 0).any()  # links along the 3-D diagonals too
    sim = q27.Sim27((20, 18, 3), 0.7, 0.0, (0, 0, 1e-5), pipe=(7.3, 9.6, 8.2))
    sim.step(3)
    assert np.isfinite(sim.u[:, ~solid]).all()
