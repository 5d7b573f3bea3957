"""Learned near-surface gradient corrector, FP64 reference: interface cells,
network features, training labels and the corrected dissipation.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module.

The paper observes that the immersed boundary method smears the velocity
gradient next to the surface, so the local dissipation there differs from
the interpolated bounce-back result (Sec. 3.2.1, Sec. 4). The
corrector is this build's addition; its readings:

* Interface cells of sphere p: fluid nodes with r_p <= |x - X_p| <
  r_p - r_d + 2 (the marker radius plus the reach of the 4-point delta).
* Fallback to the plain central difference (the cell is not corrected) when
  another sphere q is near: |x - X_q| < r_q - r_d + 2 + sqrt(3), i.e. the
  3x3x3 stencil touches q's interface band or interior, which also covers a
  gap below two spacings; or when d = |x - X_p| - r_p is outside the
  training range [d_min, d_max].
* Features (85): for the 27 offsets o (z slowest, x fastest, each -1, 0, 1)
  and the 3 components, (u(x + o) - [U_p + Omega_p x (x + o - X_p)]) / u_rms
  of the immersed-boundary field as it is; then d; then the unit normal
  (x - X_p) / |x - X_p|. Offsets are minimum-image.
* Outputs (9): the correction of the plain gradient, (G_ref - G_plain) / u_rms
  row-major in (i, j), G_ij = d_j u_i: G_plain is the central difference of
  the masked immersed-boundary field, G_ref the same operator on the paired
  bounce-back field (Sec. 3.2.1 masking). The corrected gradient is
  G_plain + u_rms y. Predicting the correction rather than G itself keeps the
  particle's rigid rotation, which the relative-velocity features cannot see,
  inside G_plain.
* Corrected dissipation: eps = 2 nu s_ij s_ij with s the symmetric part of
  the corrected G at corrected cells, the plain masked value elsewhere.

Distances follow the classification recipe of the statistics: minimum-image
offsets, squared distance ((dx dx + dy dy) + dz dz), comparisons on squared
distances against squared radii.
"""
import numpy as np

from . import stats
from .geometry import dist2

SQRT3 = float(np.sqrt(3.0))
N_FEATURES = 85


def band_outer(r, r_d):
    return r - r_d + 2.0


def exclusion_radius(r, r_d):
    return r - r_d + 2.0 + SQRT3


def interface_cells(shape, X, r, r_d, d_min, d_max):
    """(flat node indices ascending, owning sphere) of the corrected cells."""
    X = np.asarray(X, np.float64)
    r = np.asarray(r, np.float64)
    xyz = stats.node_coords(shape)
    n = len(r)
    nz_ = xyz.shape[1:]
    owner = np.full(nz_, -1, np.int64)
    zone = np.zeros(nz_, np.int64)
    for p in range(n):
        D2 = dist2(stats._offsets(X[p], xyz, shape))
        ro = band_outer(r[p], r_d)
        band = (D2 >= r[p] * r[p]) & (D2 < ro * ro)
        d = np.sqrt(D2) - r[p]
        band &= (d >= d_min) & (d <= d_max)
        owner[band] = p                        # several bands: excluded below
        re = exclusion_radius(r[p], r_d)
        zone += D2 < re * re
    keep = (owner >= 0) & (zone == 1)
    flat = np.flatnonzero(keep.ravel())
    return flat, owner.ravel()[flat]


def _node_xyz(flat, shape):
    nx, ny, _ = shape
    return np.stack([flat % nx, (flat // nx) % ny, flat // (nx * ny)], -1)


def features(u, flat, part, X, U, Om, r, u_rms, shape):
    """(n, 85) features of the cells (u: the immersed-boundary field)."""
    u = np.asarray(u, np.float64)
    nx, ny, nz = shape
    xyz = _node_xyz(flat, shape).astype(np.int64)
    Xp, Up, Wp = np.asarray(X)[part], np.asarray(U)[part], np.asarray(Om)[part]
    F = np.zeros((len(flat), N_FEATURES))
    o = 0
    for oz in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                x = (xyz[:, 0] + ox) % nx
                y = (xyz[:, 1] + oy) % ny
                z = (xyz[:, 2] + oz) % nz
                rr = np.stack([stats.min_image(x - Xp[:, 0], nx), stats.min_image(y - Xp[:, 1], ny),
                               stats.min_image(z - Xp[:, 2], nz)], -1)
                rigid = Up + np.cross(Wp, rr)
                for c in range(3):
                    F[:, 3 * o + c] = (u[c, z, y, x] - rigid[:, c]) / u_rms
                o += 1
    rr = np.stack([stats.min_image(xyz[:, 0] - Xp[:, 0], nx), stats.min_image(xyz[:, 1] - Xp[:, 1], ny),
                   stats.min_image(xyz[:, 2] - Xp[:, 2], nz)], -1)
    dist = np.sqrt(dist2(rr))
    F[:, 81] = dist - np.asarray(r)[part]
    F[:, 82:85] = rr / dist[:, None]
    return F


def gradient_at(u_masked, flat, shape):
    """(n, 9) central-difference G_ij = d_j u_i at the cells, row-major."""
    G = stats.velocity_gradient(np.asarray(u_masked, np.float64))  # (3, 3, nz, ny, nx)
    xyz = _node_xyz(flat, shape)
    return G[:, :, xyz[:, 2], xyz[:, 1], xyz[:, 0]].transpose(2, 0, 1).reshape(-1, 9)


def labels(u_pair, pair_owner, X, U, Om, flat, u_rms, shape):
    """Masked central-difference gradient of a field at the cells / u_rms
    (of the bounce-back field: the reference; of the immersed-boundary field:
    the plain gradient)."""
    um = stats.masked_velocity(u_pair, pair_owner, X, U, Om, shape)
    return gradient_at(um, flat, shape) / u_rms


def targets(labels_ref, labels_plain):
    """Training targets: the correction (G_ref - G_plain) / u_rms."""
    return np.asarray(labels_ref, np.float64) - np.asarray(labels_plain, np.float64)


def corrected_gradient(labels_plain, y, u_rms):
    """G = G_plain + u_rms y from the plain labels (G_plain / u_rms)."""
    return (np.asarray(labels_plain, np.float64) + np.asarray(y, np.float64)) * u_rms


dissipation_from_gradient = stats.dissipation_from_gradient
