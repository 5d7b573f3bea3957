"""Solid/fluid classification, boundary links and wall distances q (FP64).

Spheres (Sec. 3.1): node x is inside sphere p iff the periodic
minimum-image distance satisfies |x - X_p|^2 < r_p^2 (strict). The minimum
image uses one explicit branch per axis and the squared distance is summed
as ((dx*dx + dy*dy) + dz*dz) with no fused multiply-add, so any other
implementation that follows the same recipe classifies bit-identically.
Where spheres overlap, a node belongs to the lowest-numbered sphere
containing it (reading; the paper is silent).

Pipe wall (Sec. 2.1): solid iff (x - cx)^2 + (y - cy)^2 >= R^2.

Owner map: -1 fluid, p >= 0 sphere p, WALL for the static wall.

Boundary link (x_f, a): x_f fluid and x_f + c_a solid. q in [0, 1) is the
fraction of the link in the fluid: the smaller root of
|d + t c_a|^2 = r^2 (sphere) or its xy-projection against R (pipe), with
d = x_f - X, written in the cancellation-free form.

Fallback chain (Sec. 3.1, "when the precedent one is no longer applicable";
reading): quadratic needs x_f - c_a (and x_f - 2 c_a if q < 1/2) fluid;
otherwise linear, which needs x_f - c_a fluid if q < 1/2; otherwise the
single-node scheme. With max_order 1 the chain starts at linear.
"""
import numpy as np

from .lattice import C, CF, Q

WALL = -2
SCHEME_HALFWAY, SCHEME_LINEAR, SCHEME_QUADRATIC = 0, 1, 2


def min_image(d, L):
    """Explicit single-branch periodic wrap of d in (-L, L)."""
    d = np.asarray(d, np.float64)
    out = np.where(d > 0.5 * L, d - L, d)
    return np.where(out < -0.5 * L, out + L, out)


def sphere_offsets(X, node_xyz, shape):
    """Minimum-image offsets node - X, (..., 3) in (x, y, z)."""
    L = np.asarray(shape, np.float64)
    d = np.asarray(node_xyz, np.float64) - np.asarray(X, np.float64)
    return np.stack([min_image(d[..., k], L[k]) for k in range(3)], -1)


def dist2(d):
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


def box_nodes(X, reach, shape):
    """Integer node coordinates (x, y, z) of the periodic box
    floor(X - reach) .. ceil(X + reach) around a point, wrapped."""
    lo = np.floor(np.asarray(X) - reach).astype(int)
    hi = np.ceil(np.asarray(X) + reach).astype(int)
    ax = [np.arange(lo[k], hi[k] + 1) % shape[k] for k in range(3)]
    xs, ys, zs = np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
    pts = np.stack([xs.ravel(), ys.ravel(), zs.ravel()], -1)
    return np.unique(pts, axis=0)


def pipe_solid(shape, radius, cx, cy):
    nx, ny, nz = shape
    x = np.arange(nx, dtype=np.float64) - cx
    y = np.arange(ny, dtype=np.float64) - cy
    r2 = y[:, None] * y[:, None] + x[None, :] * x[None, :]
    return np.broadcast_to(r2 >= radius * radius, (nz, ny, nx))


def owner_map(shape, X, r, wall_solid=None):
    """Owner of every node, [z, y, x] int64."""
    nx, ny, nz = shape
    owner = np.full((nz, ny, nx), -1, np.int64)
    if wall_solid is not None:
        owner[wall_solid] = WALL
    for p in range(len(r)):
        pts = box_nodes(X[p], r[p] + 1.0, shape)
        d = sphere_offsets(X[p], pts, shape)
        inside = dist2(d) < r[p] * r[p]
        pts = pts[inside]
        cur = owner[pts[:, 2], pts[:, 1], pts[:, 0]]
        take = cur == -1
        owner[pts[take, 2], pts[take, 1], pts[take, 0]] = p
    return owner


def sphere_q(d, c, r):
    """Smaller root t of |d + t c|^2 = r^2 for an outside point heading in."""
    a = (c * c).sum(-1)
    b = (d * c).sum(-1)
    cc = dist2(d) - r * r
    return cc / (-b + np.sqrt(b * b - a * cc))


def pipe_q(dxy, cxy, R):
    """Root t in [0, 1) of |dxy + t cxy|^2 = R^2 for an inside point heading
    out (cc < 0)."""
    a = (cxy * cxy).sum(-1)
    b = (dxy * cxy).sum(-1)
    cc = (dxy[..., 0] * dxy[..., 0] + dxy[..., 1] * dxy[..., 1]) - R * R
    disc = np.sqrt(b * b - a * cc)
    return np.where(b >= 0, -cc / (b + disc), (disc - b) / np.where(a > 0, a, 1.0))


def build_links(owner, X, r, shape, max_order=2, pipe=None):
    """All boundary links. Returns a dict of arrays, one entry per link:
    xf (L, 3) int (x, y, z), a (L,) oracle direction, p (L,) owner,
    q (L,) float64, scheme (L,) int."""
    nx, ny, nz = shape
    fluid = owner == -1
    out = {k: [] for k in ("xf", "a", "p", "q", "scheme")}
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for a in range(1, Q):
        cx, cy, cz = C[a]
        own_s = np.roll(owner, shift=(-cz, -cy, -cx), axis=(0, 1, 2))     # owner at x + c_a
        hit = fluid & (own_s != -1)
        if not hit.any():
            continue
        z, y, x = zz[hit], yy[hit], xx[hit]
        p = own_s[hit]
        xf = np.stack([x, y, z], -1)
        q = np.empty(len(p))
        sph = p >= 0
        if sph.any():
            d = _offsets_many(X, p[sph], xf[sph], shape)
            q[sph] = sphere_q(d, CF[a][None, :], r[p[sph]])
        if (~sph).any():
            R, pcx, pcy = pipe
            dxy = np.stack([xf[~sph, 0] - pcx, xf[~sph, 1] - pcy], -1).astype(np.float64)
            q[~sph] = pipe_q(dxy, CF[a][None, :2].repeat(len(dxy), 0), R)
        # fallback chain on the fluid status of x_f - c_a and x_f - 2 c_a
        f1 = np.roll(fluid, shift=(cz, cy, cx), axis=(0, 1, 2))[hit]          # fluid at x - c_a
        f2 = np.roll(fluid, shift=(2 * cz, 2 * cy, 2 * cx), axis=(0, 1, 2))[hit]
        order = np.where(sph, max_order, 1)
        quad_ok = np.where(q < 0.5, f1 & f2, f1)
        lin_ok = np.where(q < 0.5, f1, True)
        scheme = np.where((order >= 2) & quad_ok, SCHEME_QUADRATIC,
                          np.where(lin_ok, SCHEME_LINEAR, SCHEME_HALFWAY))
        out["xf"].append(xf)
        out["a"].append(np.full(len(p), a))
        out["p"].append(p)
        out["q"].append(q)
        out["scheme"].append(scheme)
    if not out["a"]:
        return {"xf": np.zeros((0, 3), int), "a": np.zeros(0, int), "p": np.zeros(0, int),
                "q": np.zeros(0), "scheme": np.zeros(0, int)}
    return {k: np.concatenate(v) for k, v in out.items()}


def _offsets_many(X, p, xf, shape):
    L = np.asarray(shape, np.float64)
    d = xf.astype(np.float64) - X[p]
    return np.stack([min_image(d[:, k], L[k]) for k in range(3)], -1)
