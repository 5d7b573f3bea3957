"""Component-wise budget of the turbulent kinetic energy in the pipe, in
cylindrical coordinates (Sec. 2.2, Eq. (1a)-(1c)), FP64.

Test infrastructure: only the tests use this module.

Readings (the paper gives the equations, not their discretisation):
* Coordinates: the pipe axis runs along z through (cx, cy); for a node,
  r = |x_perp - c|, e_r = (x_perp - c) / r (e_r = e_x on the axis),
  e_theta = e_z x e_r. Fluid nodes are those with r^2 < R^2; the wall is
  masked to zero velocity as in the statistics.
* u_r = u.e_r, u_theta = u.e_theta, u_z; pressure p = rho / 3 (c_s^2 rho;
  the 1/rho of Eq. (1) is the mean density, 1 in lattice units).
* Gradients: G_ij = d_j u_i by the statistics' central differences of the
  masked field. The derivative factors of Eq. (1) are read as the physical
  cylindrical components of the velocity-gradient tensor,
  L_ab = e_a . G . e_b, e.g. L_r,theta = (1/r) du_r/dtheta - u_theta / r and
  L_theta,theta = (1/r) du_theta/dtheta + u_r / r; the strain is
  s_ab = e_a . S . e_b with S = (G + G^T) / 2. With this reading the three
  component dissipations add up to -2 nu <s'_ab s'_ab> and the pressure
  terms to <p' div u'>.
* Averages: over the nodes of each radial bin [k w, (k + 1) w) and over the
  snapshots added; a' = a - <a>, so <a'b'> = <ab> - <a><b> and
  <a'a'b'> = <a^2 b> - 2<a><ab> - <b><a^2> + 2<a>^2<b>.
* d/dr of a bin profile: central differences over the bin centres
  r_k = (k + 1/2) w, one-sided at the first and last bin; an empty bin gives
  NaN and so do the derivatives that use it.

The 38 moment sums per bin (MOMENTS) and the 13 terms (TERMS) are listed in
the order the C interface reports them.
"""
import numpy as np

from .stats import velocity_gradient

MOMENTS = (
    "count", "ur", "ut", "uz", "p",
    "Srr", "Srt", "Srz", "Stt", "Stz", "Szz",
    "Lzr", "Lzt", "Lzz", "Lrr", "Lrt", "Lrz", "Ltt", "Ltr", "Ltz",
    "uz_ur", "ur_ur", "ut_ur", "uz_uz", "ut_ut",
    "p_ur", "p_Lzz", "p_Lrr", "p_Ltt",
    "uz_Szr", "ur_Srr", "ut_Str",
    "Dz", "Dr", "Dt",
    "uz_uz_ur", "ur_ur_ur", "ut_ut_ur",
)
TERMS = ("EOz", "ETz", "EPz", "EVz", "EDz", "ETr", "EPr", "EVr", "EDr", "ETt", "EPt", "EVt", "EDt")


def cylindrical_fields(u, rho, shape, pipe):
    """Per fluid node of the pipe: bin radius r, (u_r, u_t, u_z), p, S and L
    as dicts of flat arrays, plus the Cartesian strain invariant S:S and
    p tr(G) and u_x^2 + u_y^2 for checks. u: (3, nz, ny, nx) masked."""
    nx, ny, nz = shape
    R, cx, cy = pipe
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    dx, dy = x - cx, y - cy
    r2 = dy * dy + dx * dx
    fluid = r2 < R * R
    G = velocity_gradient(np.asarray(u, np.float64))          # (3, 3, nz, ny, nx)
    r = np.sqrt(r2[fluid])
    safe = np.where(r > 0.0, r, 1.0)
    er = np.stack([np.where(r > 0.0, dx[fluid] / safe, 1.0), np.where(r > 0.0, dy[fluid] / safe, 0.0),
                   np.zeros_like(r)], 1)                     # (n, 3)
    et = np.stack([-er[:, 1], er[:, 0], np.zeros_like(r)], 1)
    ez = np.zeros_like(er)
    ez[:, 2] = 1.0
    B = np.stack([er, et, ez], 1)                            # rows e_r, e_t, e_z: (n, 3, 3)
    Gf = np.moveaxis(G[:, :, fluid], -1, 0)                  # (n, 3, 3)
    uf = np.moveaxis(np.asarray(u, np.float64)[:, fluid], -1, 0)
    L = np.einsum("nai,nij,nbj->nab", B, Gf, B)              # L_ab = e_a . G . e_b
    S = 0.5 * (L + np.swapaxes(L, 1, 2))
    uc = np.einsum("nai,ni->na", B, uf)
    Sc = 0.5 * (Gf + np.swapaxes(Gf, 1, 2))
    out = dict(r=r, ur=uc[:, 0], ut=uc[:, 1], uz=uc[:, 2], p=np.asarray(rho, np.float64)[fluid] / 3.0)
    names = ("r", "t", "z")
    for a in range(3):
        for b in range(3):
            out["L" + names[a] + names[b]] = L[:, a, b]
            out["S" + names[a] + names[b]] = S[:, a, b]
    out["SS_cart"] = (Sc * Sc).sum((1, 2))
    out["p_trG"] = out["p"] * np.trace(Gf, axis1=1, axis2=2)
    out["uxuy2"] = uf[:, 0] ** 2 + uf[:, 1] ** 2
    return out


def moment_sums(f, width, nbins):
    """(38, nbins) sums of MOMENTS over the nodes of each bin."""
    q = {
        "count": np.ones_like(f["r"]), "ur": f["ur"], "ut": f["ut"], "uz": f["uz"], "p": f["p"],
        "Srr": f["Srr"], "Srt": f["Srt"], "Srz": f["Srz"], "Stt": f["Stt"], "Stz": f["Stz"], "Szz": f["Szz"],
        "Lzr": f["Lzr"], "Lzt": f["Lzt"], "Lzz": f["Lzz"], "Lrr": f["Lrr"], "Lrt": f["Lrt"], "Lrz": f["Lrz"],
        "Ltt": f["Ltt"], "Ltr": f["Ltr"], "Ltz": f["Ltz"],
        "uz_ur": f["uz"] * f["ur"], "ur_ur": f["ur"] * f["ur"], "ut_ur": f["ut"] * f["ur"],
        "uz_uz": f["uz"] * f["uz"], "ut_ut": f["ut"] * f["ut"],
        "p_ur": f["p"] * f["ur"], "p_Lzz": f["p"] * f["Lzz"], "p_Lrr": f["p"] * f["Lrr"], "p_Ltt": f["p"] * f["Ltt"],
        "uz_Szr": f["uz"] * f["Szr"], "ur_Srr": f["ur"] * f["Srr"], "ut_Str": f["ut"] * f["Str"],
        "Dz": f["Szr"] * f["Lzr"] + f["Szt"] * f["Lzt"] + f["Szz"] * f["Lzz"],
        "Dr": f["Srr"] * f["Lrr"] + f["Srt"] * f["Lrt"] + f["Srz"] * f["Lrz"],
        "Dt": f["Stt"] * f["Ltt"] + f["Str"] * f["Ltr"] + f["Stz"] * f["Ltz"],
        "uz_uz_ur": f["uz"] * f["uz"] * f["ur"], "ur_ur_ur": f["ur"] ** 3, "ut_ut_ur": f["ut"] * f["ut"] * f["ur"],
    }
    b = np.floor(f["r"] / width).astype(np.int64)
    keep = b < nbins
    out = np.zeros((len(MOMENTS), nbins))
    for i, name in enumerate(MOMENTS):
        out[i] = np.bincount(b[keep], weights=q[name][keep], minlength=nbins)[:nbins]
    return out


def _ddr(f, w):
    """d f / dr over bin centres: central, one-sided at the ends."""
    d = np.empty_like(f)
    if len(f) == 1:
        d[:] = np.nan
        return d
    d[1:-1] = (f[2:] - f[:-2]) / (2.0 * w)
    d[0] = (f[1] - f[0]) / w
    d[-1] = (f[-1] - f[-2]) / w
    return d


def budget_terms(M, width, nu):
    """(13, nbins) TERMS from accumulated moment sums M (38, nbins)."""
    M = np.asarray(M, np.float64)
    n = M[0]
    with np.errstate(invalid="ignore", divide="ignore"):
        m = {name: M[i] / n for i, name in enumerate(MOMENTS)}
    rk = (np.arange(M.shape[1]) + 0.5) * width

    def cyl_div(f):  # (1/r) d(r f)/dr
        return _ddr(rk * f, width) / rk

    c_zr = m["uz_ur"] - m["uz"] * m["ur"]
    Tz = 0.5 * (m["uz_uz_ur"] - 2.0 * m["uz"] * m["uz_ur"] - m["ur"] * m["uz_uz"] + 2.0 * m["uz"] ** 2 * m["ur"])
    Tr = 0.5 * (m["ur_ur_ur"] - 3.0 * m["ur"] * m["ur_ur"] + 2.0 * m["ur"] ** 3)
    Tt = 0.5 * (m["ut_ut_ur"] - 2.0 * m["ut"] * m["ut_ur"] - m["ur"] * m["ut_ut"] + 2.0 * m["ut"] ** 2 * m["ur"])
    E = {
        "EOz": -c_zr * _ddr(m["uz"], width),
        "ETz": -cyl_div(Tz),
        "EPz": m["p_Lzz"] - m["p"] * m["Lzz"],
        "EVz": 2.0 * nu * cyl_div(m["uz_Szr"] - m["uz"] * m["Srz"]),
        "EDz": -2.0 * nu * (m["Dz"] - (m["Srz"] * m["Lzr"] + m["Stz"] * m["Lzt"] + m["Szz"] * m["Lzz"])),
        "ETr": -cyl_div(Tr),
        "EPr": -_ddr(m["p_ur"] - m["ur"] * m["p"], width) + (m["p_Lrr"] - m["p"] * m["Lrr"]),
        "EVr": 2.0 * nu * cyl_div(m["ur_Srr"] - m["ur"] * m["Srr"]),
        "EDr": -2.0 * nu * (m["Dr"] - (m["Srr"] * m["Lrr"] + m["Srt"] * m["Lrt"] + m["Srz"] * m["Lrz"])),
        "ETt": -cyl_div(Tt),
        "EPt": m["p_Ltt"] - m["p"] * m["Ltt"],
        "EVt": 2.0 * nu * cyl_div(m["ut_Str"] - m["ut"] * m["Srt"]),
        "EDt": -2.0 * nu * (m["Dt"] - (m["Stt"] * m["Ltt"] + m["Srt"] * m["Ltr"] + m["Stz"] * m["Ltz"])),
    }
    return np.stack([E[t] for t in TERMS])


def add_snapshot(M, u, rho, shape, pipe, width):
    """Adds one snapshot's moment sums to M (38, nbins) in place."""
    M += moment_sums(cylindrical_fields(u, rho, shape, pipe), width, M.shape[1])
    return M
