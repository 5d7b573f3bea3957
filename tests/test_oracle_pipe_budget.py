"""Pins of the FP64 oracle for the pipe's component TKE budget (Eq. (1a)-(1c)):
rotation invariants against the Cartesian strain, closed forms for rigid
rotation, radial stretching and a travelling-wave fluctuation, and the
radial differences."""
import numpy as np
import pytest

from oracle import pipe_budget as pb

SHAPE = (24, 22, 16)
PIPE = (9.3, 11.4, 10.7)


def _coords():
    nx, ny, nz = SHAPE
    z, y, x = np.meshgrid(np.arange(nz, dtype=float), np.arange(ny, dtype=float), np.arange(nx, dtype=float),
                          indexing="ij")
    return x - PIPE[1], y - PIPE[2], z


def _masked(u):
    R = PIPE[0]
    xp, yp, _ = _coords()
    wall = xp * xp + yp * yp >= R * R
    u = np.array(u, float)
    u[:, wall] = 0.0
    return u


def _interior(f, margin=1.5):
    return f["r"] < PIPE[0] - margin


def test_rotation_invariants_random_field():
    rng = np.random.default_rng(4)
    nx, ny, nz = SHAPE
    u = _masked(rng.normal(scale=0.05, size=(3, nz, ny, nx)))
    rho = 1.0 + rng.normal(scale=0.01, size=(nz, ny, nx))
    f = pb.cylindrical_fields(u, rho, SHAPE, PIPE)
    M = pb.moment_sums(f, 0.5, 19)
    b = np.floor(f["r"] / 0.5).astype(int)
    ss = np.bincount(b, weights=f["SS_cart"], minlength=19)[:19]
    ptr = np.bincount(b, weights=f["p_trG"], minlength=19)[:19]
    uu = np.bincount(b, weights=f["uxuy2"], minlength=19)[:19]
    i = {n: k for k, n in enumerate(pb.MOMENTS)}
    scale = np.abs(ss).max()
    assert np.abs(M[i["Dz"]] + M[i["Dr"]] + M[i["Dt"]] - ss).max() <= 1e-12 * scale
    assert np.abs(M[i["p_Lzz"]] + M[i["p_Lrr"]] + M[i["p_Ltt"]] - ptr).max() <= 1e-12 * np.abs(ptr).max()
    assert np.abs(M[i["ur_ur"]] + M[i["ut_ut"]] - uu).max() <= 1e-12 * np.abs(uu).max()
    # every fluid node counted once
    assert M[0].sum() == len(f["r"])


def test_rigid_rotation_has_no_strain_and_signed_curvature_terms():
    om = 0.013
    xp, yp, z = _coords()
    u = _masked(np.stack([-om * yp, om * xp, np.zeros_like(z)]))
    f = pb.cylindrical_fields(u, np.ones(u.shape[1:]), SHAPE, PIPE)
    k = _interior(f)
    for s in ("Srr", "Srt", "Srz", "Stt", "Stz", "Szz"):
        assert np.abs(f[s][k]).max() < 1e-15
    assert np.allclose(f["Lrt"][k], -om, rtol=0, atol=1e-15)   # (1/r) du_r/dtheta - u_theta/r
    assert np.allclose(f["Ltr"][k], om, rtol=0, atol=1e-15)    # du_theta/dr
    assert np.allclose(f["ut"][k], om * f["r"][k], rtol=0, atol=1e-15)
    assert np.abs(f["ur"][k]).max() < 1e-15


def test_radial_stretch_closed_form():
    a, c = 0.004, 0.02
    xp, yp, z = _coords()
    u = _masked(np.stack([a * xp, a * yp, np.full_like(z, c)]))
    f = pb.cylindrical_fields(u, np.ones(u.shape[1:]), SHAPE, PIPE)
    k = _interior(f)
    for name, v in (("Lrr", a), ("Ltt", a), ("Lzz", 0.0), ("Srt", 0.0), ("Lrt", 0.0), ("Ltr", 0.0)):
        assert np.allclose(f[name][k], v, rtol=0, atol=1e-16), name
    assert np.allclose(f["ur"][k], a * f["r"][k], rtol=0, atol=1e-15)
    M = pb.moment_sums({q: v[k] for q, v in f.items()}, 0.5, 16)
    i = {n: j for j, n in enumerate(pb.MOMENTS)}
    assert np.allclose(M[i["Dr"]], a * a * M[0], rtol=1e-12, atol=0)
    assert np.allclose(M[i["Dt"]], a * a * M[0], rtol=1e-12, atol=0)
    assert np.abs(M[i["Dz"]]).max() < 1e-18


def test_wave_fluctuation_production_and_pressure_work():
    """u_z = U(r) + e sin(kz), u_r = e sin(kz), p = p0 + d cos(kz): the
    covariance <u_z'u_r'> is e^2/2 in every bin (the radial profile and the
    wave are independent), so E_Oz = -(e^2/2) dU/dr, and
    E_Pz = <p' d_z u_z'> = d e sin(k) / 2 with the central difference."""
    nx, ny, nz = SHAPE
    e, dd, A = 1e-3, 2e-3, 2e-4
    k = 2 * np.pi * 3 / nz
    xp, yp, z = _coords()
    r = np.sqrt(xp * xp + yp * yp)
    s = np.sin(k * z)
    ur = e * s
    er = np.stack([np.where(r > 0, xp / np.where(r > 0, r, 1), 1.0), np.where(r > 0, yp / np.where(r > 0, r, 1), 0.0)])
    U = A * (PIPE[0] ** 2 - r * r)
    u = _masked(np.stack([ur * er[0], ur * er[1], U + e * s]))
    rho = 3.0 * (1.0 / 3.0 + dd * np.cos(k * z))
    f = pb.cylindrical_fields(u, rho, SHAPE, PIPE)
    w = 1.0
    nb = int(np.ceil(PIPE[0] / w))
    M = pb.moment_sums(f, w, nb)
    T = pb.budget_terms(M, w, nu=0.01)
    t = {n: j for j, n in enumerate(pb.TERMS)}
    ok = np.arange(nb) < int((PIPE[0] - 1.5) / w) - 1  # bins whose stencils and neighbours stay inside
    # the bin means of U(r) from the fluid nodes, differenced like the oracle
    b = np.floor(f["r"] / w).astype(int)
    Ubar = np.bincount(b, weights=A * (PIPE[0] ** 2 - f["r"] ** 2), minlength=nb)[:nb] / M[0]
    dU = np.empty(nb)
    dU[1:-1] = (Ubar[2:] - Ubar[:-2]) / (2 * w)
    dU[0] = (Ubar[1] - Ubar[0]) / w
    dU[-1] = (Ubar[-1] - Ubar[-2]) / w
    assert np.allclose(T[t["EOz"]][ok], -(e * e / 2) * dU[ok], rtol=1e-9, atol=0)
    assert np.allclose(T[t["EPz"]][ok], dd * e * np.sin(k) / 2, rtol=1e-9, atol=0)


def test_radial_differences_exact_for_quadratics():
    w = 0.5
    rk = (np.arange(12) + 0.5) * w
    f = 3.0 - 0.2 * rk + 0.07 * rk * rk
    d = pb._ddr(f, w)
    assert np.allclose(d[1:-1], -0.2 + 0.14 * rk[1:-1], rtol=0, atol=1e-14)
    # one-sided ends are the secant slope
    assert np.isclose(d[0], (f[1] - f[0]) / w)


def test_empty_bins_give_nan():
    M = np.zeros((len(pb.MOMENTS), 4))
    M[0, 1:] = 10.0
    T = pb.budget_terms(M, 0.5, 0.01)
    assert np.isnan(T[:, 0]).all()
