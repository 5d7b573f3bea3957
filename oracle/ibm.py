"""Immersed boundary method pieces (Sec. 2.1, Sec. 3.1; FP64).

* Peskin's 4-point regularised delta function (Peskin 2002), named in
  Sec. 2.1:
      phi(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4r^2)) / 8      |r| <= 1
             = (5 - 2|r| - sqrt(-7 + 12|r| - 4r^2)) / 8    1 <= |r| <= 2
             = 0                                           otherwise
  delta(x) = phi(x) phi(y) phi(z); the support of a point X is the 4x4x4
  block of nodes floor(X_k) - 1 .. floor(X_k) + 2 per axis.
* Lagrangian markers on a sphere (reading; the paper fixes only that the
  marker volume is close to the cell volume, Sec. 2.1): retracted radius
  r_L = r - r_d (r_d = 0 Uhlmann, 0.4 Breugem), count
  N_L = round(pi (12 r_L^2 + 1) / 3), volume
  dV = 4/3 pi ((r_L + 1/2)^3 - (r_L - 1/2)^3) / N_L, directions on a
  Fibonacci lattice z_k = 1 - (2k+1)/N_L, phi_k = k pi (3 - sqrt 5).
* Pipe markers (Sec. 2.1): rings at every integer z with
  N_theta = round(2 pi r_L) markers, dV = 2 pi r_L / N_theta; the
  retraction moves the ring into the wall, r_L = R + r_d (reading).
* Multi-direct forcing (Sec. 2.1 and Sec. 3.1: the prediction plus two
  iterations): every pass interpolates U_l from the current velocity at all
  markers, sets dF_l = 2 (U_d - U_l) (factor 2 from the half-force velocity,
  reference density 1; reading), spreads dF_l delta dV into the node force
  and corrects the velocity by the spread force / (2 rho).
* Kempe et al. 2012 inner-fluid inertia (Sec. 3.1): cell solid fraction
  alpha = sum_m (-phi_m) H(-phi_m) / sum_m |phi_m| over the 8 corners of the
  unit cell around a node, phi_m = |x_m - X| - r the signed distance.
"""
import numpy as np

from .geometry import _offsets_many, dist2, min_image


def peskin_phi(r):
    a = np.abs(np.asarray(r, np.float64))
    out = np.zeros_like(a)
    inner = a <= 1.0
    outer = (a > 1.0) & (a < 2.0)
    out[inner] = (3.0 - 2.0 * a[inner] + np.sqrt(1.0 + 4.0 * a[inner] - 4.0 * a[inner] ** 2)) / 8.0
    ao = a[outer]
    out[outer] = (5.0 - 2.0 * ao - np.sqrt(np.maximum(-7.0 + 12.0 * ao - 4.0 * ao ** 2, 0.0))) / 8.0
    return out


def sphere_marker_count(r_l):
    return int(round(np.pi * (12.0 * r_l * r_l + 1.0) / 3.0))


def sphere_marker_volume(r_l, n):
    return (4.0 / 3.0) * np.pi * ((r_l + 0.5) ** 3 - (r_l - 0.5) ** 3) / n


def fibonacci_directions(n):
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    phi = k * (np.pi * (3.0 - np.sqrt(5.0)))
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], -1)


def sphere_markers(X, r, r_d, shape):
    """Marker positions (wrapped into the box), their particle, offsets from
    the centre and volumes for all spheres."""
    L = np.asarray(shape, np.float64)
    pos, owner, arm, vol = [], [], [], []
    for p in range(len(r)):
        r_l = r[p] - r_d
        n = sphere_marker_count(r_l)
        dirs = fibonacci_directions(n)
        a = r_l * dirs
        xl = X[p] + a
        xl = np.where(xl >= L, xl - L, xl)
        xl = np.where(xl < 0.0, xl + L, xl)
        pos.append(xl)
        owner.append(np.full(n, p))
        arm.append(a)
        vol.append(np.full(n, sphere_marker_volume(r_l, n)))
    if not pos:
        return np.zeros((0, 3)), np.zeros(0, int), np.zeros((0, 3)), np.zeros(0)
    return np.concatenate(pos), np.concatenate(owner), np.concatenate(arm), np.concatenate(vol)


def pipe_markers(R, r_d, cx, cy, nz):
    r_l = R + r_d
    n = int(round(2.0 * np.pi * r_l))
    th = 2.0 * np.pi * np.arange(n) / n
    ring = np.stack([cx + r_l * np.cos(th), cy + r_l * np.sin(th)], -1)
    pos = np.concatenate([np.column_stack([ring, np.full(n, float(z))]) for z in range(nz)])
    return pos, np.full(len(pos), 2.0 * np.pi * r_l / n)


def stencils(xl, shape):
    """Nodes (M, 64, 3) and weights (M, 64) of the delta around every
    marker position xl (M, 3)."""
    xl = np.atleast_2d(np.asarray(xl, np.float64))
    base = np.floor(xl).astype(np.int64) - 1                         # (M, 3)
    off = np.arange(4)
    idx = base[:, :, None] + off[None, None, :]                       # (M, 3, 4)
    w = peskin_phi(xl[:, :, None] - idx)                              # (M, 3, 4)
    wgt = (w[:, 0, :, None, None] * w[:, 1, None, :, None]) * w[:, 2, None, None, :]
    ix = np.broadcast_to(idx[:, 0, :, None, None], wgt.shape) % shape[0]
    iy = np.broadcast_to(idx[:, 1, None, :, None], wgt.shape) % shape[1]
    iz = np.broadcast_to(idx[:, 2, None, None, :], wgt.shape) % shape[2]
    nodes = np.stack([ix, iy, iz], -1).reshape(len(xl), 64, 3)
    return nodes, wgt.reshape(len(xl), 64)


def interpolate(u, xl, shape):
    """U_l = sum_x delta(x - X_l) u(x) for every marker; u [3, z, y, x]."""
    nodes, w = stencils(xl, shape)
    vals = u[:, nodes[..., 2], nodes[..., 1], nodes[..., 0]]          # (3, M, 64)
    return (vals * w[None]).sum(-1).T


def spread(F_l, dV, xl, shape):
    """f(x) = sum_l F_l delta(x - X_l) dV_l on the grid, [3, z, y, x]."""
    nx, ny, nz = shape
    f = np.zeros((3, nz, ny, nx))
    nodes, w = stencils(xl, shape)
    flat = (nodes[..., 2] * ny + nodes[..., 1]) * nx + nodes[..., 0]  # (M, 64)
    for k in range(3):
        contrib = (F_l[:, k] * dV)[:, None] * w
        np.add.at(f[k].reshape(-1), flat.ravel(), contrib.ravel())
    return f


def multi_direct_forcing(u_star, rho, xl, U_d, dV, passes, shape):
    """Returns (node force f_IB [3, z, y, x], corrected velocity, marker
    force F_l (markers, 3) summed over passes)."""
    u = u_star.copy()
    f_ib = np.zeros_like(u_star)
    F_l = np.zeros((len(xl), 3))
    for _ in range(passes):
        U_l = interpolate(u, xl, shape)
        dF = 2.0 * (U_d - U_l)
        F_l += dF
        df = spread(dF, dV, xl, shape)
        f_ib += df
        u = u + df / (2.0 * rho)
    return f_ib, u, F_l


_CORNERS = np.array([[sx, sy, sz] for sx in (-0.5, 0.5) for sy in (-0.5, 0.5) for sz in (-0.5, 0.5)])


def solid_fraction(X, r, nodes, shape):
    """Kempe alpha at integer nodes (M, 3) for one sphere."""
    d = _offsets_many(np.asarray(X)[None], np.zeros(len(nodes), int), nodes, shape)
    num = np.zeros(len(nodes))
    den = np.zeros(len(nodes))
    for c in _CORNERS:
        phi = np.sqrt(dist2(d + c)) - r
        num += np.where(phi < 0.0, -phi, 0.0)
        den += np.abs(phi)
    return np.where(den > 0, num / den, 0.0)


def inner_integrals(u, X, r, shape):
    """I_u = sum alpha u and I_L = sum alpha (x - X) x u per sphere over the
    cells with alpha > 0, for u [3, z, y, x]."""
    from .geometry import box_nodes
    n = len(r)
    Iu = np.zeros((n, 3))
    IL = np.zeros((n, 3))
    for p in range(n):
        nodes = box_nodes(X[p], r[p] + 1.0, shape)
        alpha = solid_fraction(X[p], r[p], nodes, shape)
        keep = alpha > 0
        nodes = nodes[keep]
        alpha = alpha[keep]
        uu = u[:, nodes[:, 2], nodes[:, 1], nodes[:, 0]].T
        arm = _offsets_many(X[p][None], np.zeros(len(nodes), int), nodes, shape)
        Iu[p] = (alpha[:, None] * uu).sum(0)
        IL[p] = (alpha[:, None] * np.cross(arm, uu)).sum(0)
    return Iu, IL


__all__ = ["peskin_phi", "sphere_marker_count", "sphere_marker_volume", "fibonacci_directions",
           "sphere_markers", "pipe_markers", "stencils", "interpolate", "spread", "multi_direct_forcing",
           "solid_fraction", "inner_integrals", "min_image"]
