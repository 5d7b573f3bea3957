"""Flow and particle statistics (FP64): kinetic energy, dissipation, local
profiles over the distance to the nearest surface, particle energies, and
host energy spectra.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module.

* Kinetic energy (Sec. 3.2.1): 1/2 <|u|^2> over the lattice.
* Dissipation rate (Sec. 3.2.1): eps = 2 nu <s_ij s_ij>, s_ij = (d_i u_j +
  d_j u_i) / 2. The paper evaluates global statistics spectrally; here the
  velocity gradient is the second-order central difference on the periodic
  lattice, d_x u(x) = (u(x + e_x) - u(x - e_x)) / 2 (reading; the GPU path
  uses the same operator, so the two are comparable).
* Masking (Sec. 3.2.1): inside a particle the velocity is replaced by the
  rigid-body motion U + Omega x (x - X) before averaging and differencing;
  inside the pipe wall by zero. Unmasked values use the lattice field as it
  is (meaningful for the immersed boundary method, whose interior fluid
  evolves, and for runs without particles).
* Local profiles (Sec. 3.2.1): fluid nodes binned by their distance
  to the nearest surface, d(x) = min over particles of (|x - X_p| - r_p) and,
  with a pipe, R - |x_perp - c|; every node is counted once, in the bin
  floor(d / width). Per bin: node count and the sums of 1/2 |u|^2, eps (of
  the masked field), u_z and u_z^2 (the pipe's radial mean and rms), and the
  corrected eps.
* Corrected dissipation (optional): at the cells a gradient corrector
  handles, eps from the symmetric part of the supplied gradient instead of
  the central difference; eps_fluid_corrected and a sixth histogram row
  (sum of corrected eps) report it, equal to the plain values without one.
* Particle energies (Sec. 3.2.2): 1/2 sum m |U|^2 and 1/2 sum I |Omega|^2 with
  m = rho_p 4/3 pi r^3, I = 2/5 m r^2.
* Spectra (Sec. 3.2.1, Table 2): E(k) by integer-shell binning of 1/2 |u_hat|^2,
  D(k) = 2 nu k^2 E(k).

A node is inside sphere p iff its minimum-image squared distance (summed as
((dx dx + dy dy) + dz dz)) is below r_p^2; the lowest-numbered sphere owns a
node inside several.

Fields are (3, nz, ny, nx); positions (np, 3) in (x, y, z).
"""
import numpy as np

from .geometry import dist2, min_image

BIN_WIDTH = 0.25  # distance bins of a quarter lattice spacing (Sec. 3.2.1)


def node_coords(shape):
    """(3, nz, ny, nx) FP64 coordinates (x, y, z) of every node."""
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return np.stack([x, y, z])


def _offsets(Xp, xyz, shape):
    return np.stack([min_image(xyz[k] - Xp[k], float(shape[k])) for k in range(3)], -1)


def classify(shape, X, r, pipe=None, width=BIN_WIDTH, nbins=32):
    """Per node: owner (-1 fluid, p >= 0 sphere, -2 pipe wall) and the bin of
    the distance to the nearest surface (-1 if not binned: solid, or d at or
    beyond nbins * width)."""
    nx, ny, nz = shape
    xyz = node_coords(shape)
    owner = np.full((nz, ny, nx), -1, np.int64)
    dmin = np.full((nz, ny, nx), np.inf)
    if pipe is not None:
        R, cx, cy = pipe
        dx = xyz[0] - cx
        dy = xyz[1] - cy
        r2 = dy * dy + dx * dx
        owner[r2 >= R * R] = -2
        dmin = np.minimum(dmin, R - np.sqrt(r2))
    for p in range(len(r)):
        d2 = dist2(_offsets(X[p], xyz, shape))
        inside = (d2 < r[p] * r[p]) & (owner == -1)
        owner[inside] = p
        dmin = np.minimum(dmin, np.sqrt(d2) - r[p])
    fluid = owner == -1
    b = np.full((nz, ny, nx), -1, np.int64)
    ok = fluid & (dmin < nbins * width)
    b[ok] = np.floor(dmin[ok] / width).astype(np.int64)
    return owner, b


def masked_velocity(u, owner, X, U, Om, shape):
    """u with the rigid-body motion inside particles and zero in the wall."""
    um = np.array(u, np.float64, copy=True)
    xyz = node_coords(shape)
    um[:, owner == -2] = 0.0
    for p in range(len(X)):
        sel = owner == p
        if not sel.any():
            continue
        d = _offsets(X[p], xyz[:, sel], shape)        # (n, 3)
        w = np.cross(np.broadcast_to(Om[p], d.shape), d)
        um[:, sel] = (U[p][None, :] + w).T
    return um


def velocity_gradient(u):
    """G[i, j] = d_j u_i by periodic central differences; (3, 3, nz, ny, nx)."""
    G = np.empty((3, 3) + u.shape[1:])
    for j, ax in enumerate((3, 2, 1)):  # x, y, z axes of (3, nz, ny, nx)
        G[:, j] = 0.5 * (np.roll(u, -1, axis=ax) - np.roll(u, 1, axis=ax))
    return G


def dissipation_field(u, nu):
    """eps(x) = 2 nu s_ij s_ij with s = (G + G^T) / 2."""
    G = velocity_gradient(u)
    S = 0.5 * (G + G.transpose(1, 0, 2, 3, 4))
    return 2.0 * nu * (S * S).sum((0, 1))


def dissipation_from_gradient(G, nu):
    """eps = 2 nu s_ij s_ij for rows of 9 gradient entries G_ij = d_j u_i."""
    G = np.asarray(G, np.float64).reshape(-1, 3, 3)
    S = 0.5 * (G + G.transpose(0, 2, 1))
    return 2.0 * nu * (S * S).sum((1, 2))


def statistics(u, rho, nu, shape, X=None, U=None, Om=None, r=None, rho_p=None, pipe=None,
               width=BIN_WIDTH, nbins=32, corrected=None):
    """All statistics of one snapshot; means are over the N nodes (masked and
    raw) or the N_f fluid nodes (the *_fluid entries). corrected: optional
    (flat node indices, (n, 9) gradients) of corrected fluid cells."""
    n = 0 if r is None else len(r)
    X = np.zeros((0, 3)) if n == 0 else np.asarray(X, np.float64)
    U = np.zeros((n, 3)) if U is None else np.asarray(U, np.float64)
    Om = np.zeros((n, 3)) if Om is None else np.asarray(Om, np.float64)
    r = np.zeros(0) if n == 0 else np.asarray(r, np.float64)
    rho_p = np.ones(n) if rho_p is None else np.asarray(rho_p, np.float64)
    u = np.asarray(u, np.float64)
    rho = np.asarray(rho, np.float64)
    owner, b = classify(shape, X, r, pipe, width, nbins)
    fluid = owner == -1
    um = masked_velocity(u, owner, X, U, Om, shape)
    ke_raw = 0.5 * (u * u).sum(0)
    ke_m = 0.5 * (um * um).sum(0)
    eps_raw = dissipation_field(u, nu)
    eps_m = dissipation_field(um, nu)
    N = u[0].size
    nf = int(fluid.sum())
    m = rho_p * (4.0 / 3.0) * np.pi * r ** 3
    I = 0.4 * m * r ** 2
    out = dict(
        n_nodes=N, n_fluid=nf,
        mass=rho[fluid].sum(),
        momentum=np.array([(rho * u[k])[fluid].sum() for k in range(3)]),
        ke_raw=ke_raw.sum() / N, ke_masked=ke_m.sum() / N, ke_fluid=ke_raw[fluid].sum() / max(nf, 1),
        eps_raw=eps_raw.sum() / N, eps_masked=eps_m.sum() / N, eps_fluid=eps_m[fluid].sum() / max(nf, 1),
        umax=np.sqrt((u * u).sum(0)[fluid].max()) if nf else 0.0,
        bulk_u=u[2][fluid].sum() / max(nf, 1),
        particle_ke=0.5 * (m * (U * U).sum(1)).sum(),
        particle_ke_rot=0.5 * (I * (Om * Om).sum(1)).sum(),
    )
    eps_c = eps_m.copy()
    if corrected is not None and len(corrected[0]):
        flat, G = corrected
        eps_c.reshape(-1)[np.asarray(flat)] = dissipation_from_gradient(G, nu)
        out["n_corrected"] = len(flat)
    else:
        out["n_corrected"] = 0
    out["eps_fluid_corrected"] = eps_c[fluid].sum() / max(nf, 1)
    hist = np.zeros((6, nbins))
    sel = b >= 0
    bb = b[sel]
    hist[0] = np.bincount(bb, minlength=nbins)[:nbins]
    hist[1] = np.bincount(bb, weights=ke_raw[sel], minlength=nbins)[:nbins]
    hist[2] = np.bincount(bb, weights=eps_m[sel], minlength=nbins)[:nbins]
    hist[3] = np.bincount(bb, weights=u[2][sel], minlength=nbins)[:nbins]
    hist[4] = np.bincount(bb, weights=(u[2] * u[2])[sel], minlength=nbins)[:nbins]
    hist[5] = np.bincount(bb, weights=eps_c[sel], minlength=nbins)[:nbins]
    out["hist"] = hist
    return out


def energy_spectrum(u, kmax=None):
    """E(k) for integer shells k - 1/2 <= |k| < k + 1/2, k = 0 .. kmax (default:
    every shell, so sum E = 1/2 <|u|^2>)."""
    u = np.asarray(u, np.float64)
    nz, ny, nx = u.shape[1:]
    uh = np.fft.fftn(u, axes=(1, 2, 3)) / (nx * ny * nz)
    e = 0.5 * (np.abs(uh) ** 2).sum(0)
    kz = np.fft.fftfreq(nz, 1.0 / nz)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    kx = np.fft.fftfreq(nx, 1.0 / nx)
    kk = np.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    shell = np.floor(kk + 0.5).astype(np.int64)
    top = int(shell.max()) if kmax is None else int(kmax)
    E = np.bincount(shell.ravel(), weights=e.ravel(), minlength=top + 1)[:top + 1]
    return np.arange(top + 1, dtype=np.float64), E


def dissipation_spectrum(k, E, nu):
    """D(k) = 2 nu k^2 E(k)."""
    return 2.0 * nu * k * k * E
