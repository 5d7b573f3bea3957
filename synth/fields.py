"""Seeded initial velocity fields.

* Decaying isotropic turbulence: a random-phase, solenoidal, band-limited
  Fourier field with shell spectrum E(k) proportional to k^4 exp(-2 (k/k0)^2)
  (k in box units), scaled to a prescribed component r.m.s. The same
  coefficients can be evaluated on any grid size or at single points, so a
  large lattice and a sampled check of it see the same continuous field.
* Pipe: a parabolic axial profile plus iid uniform perturbations.

Node i sits at coordinate i; the box length along an axis is the node count.
Arrays are laid out [component, z, y, x] (x fastest), float64 unless a dtype
is given.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class HitSpectrum:
    """Hermitian Fourier coefficients of a real periodic velocity field.

    k : (M, 3) int wave vectors (box units), the full ball |k| <= kcut
    b : (M, 3) complex amplitudes with b(-k) = conj(b(k)) and k . b(k) = 0
    The field is u(x) = sum_k b_k exp(2 pi i k . x / L) on a box of side L.
    """
    k: np.ndarray
    b: np.ndarray
    kcut: int


def hit_spectrum(seed: int, u_rms: float, k0: float = 4.0, kcut: int = 14,
                 power: float = 4.0) -> HitSpectrum:
    """Draw the random-phase spectrum.

    Each wave vector gets a complex Gaussian 3-vector, projected onto the plane
    normal to k (divergence free), scaled so that shell energy follows
    E(k) ~ k^power exp(-2 (k/k0)^2), then Hermitian-symmetrised and rescaled so
    that <u_x^2> = <u_y^2> = <u_z^2> = u_rms^2 on average (Parseval).
    """
    rng = np.random.default_rng(seed)
    r = np.arange(-kcut, kcut + 1)
    kk = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    kmag2 = (kk * kk).sum(1)
    keep = (kmag2 >= 1) & (kmag2 <= kcut * kcut)
    kk = kk[keep]
    kmag = np.sqrt((kk * kk).sum(1).astype(np.float64))
    draw = rng.standard_normal((kk.shape[0], 3, 2))
    a = draw[..., 0] + 1j * draw[..., 1]
    kf = kk.astype(np.float64)
    a = a - kf * ((a * kf).sum(1) / (kmag * kmag))[:, None]
    shell = kmag ** power * np.exp(-2.0 * (kmag / k0) ** 2)
    a *= np.sqrt(shell / (4.0 * np.pi * kmag * kmag))[:, None]
    # Hermitian symmetrisation: b(k) = (a(k) + conj(a(-k))) / 2.
    index = {tuple(v): i for i, v in enumerate(kk)}
    neg = np.array([index[(-v[0], -v[1], -v[2])] for v in kk])
    b = 0.5 * (a + np.conj(a[neg]))
    energy = (np.abs(b) ** 2).sum()          # = <|u|^2>
    b *= np.sqrt(3.0 * u_rms * u_rms / energy)
    return HitSpectrum(k=kk, b=b, kcut=kcut)


def _dense_cube(spec: HitSpectrum, comp: int) -> np.ndarray:
    K = spec.kcut
    cube = np.zeros((2 * K + 1,) * 3, np.complex128)
    cube[spec.k[:, 0] + K, spec.k[:, 1] + K, spec.k[:, 2] + K] = spec.b[:, comp]
    return cube


def hit_field(spec: HitSpectrum, shape, dtype=np.float64, zchunk: int = 32):
    """Evaluate the field on a grid of shape (nx, ny, nz).

    Separable inverse transform over the band-limited support, so the cost is
    O(n^3 (2 kcut + 1)) and no full-size FFT buffer is needed.
    Returns u[3, nz, ny, nx].
    """
    nx, ny, nz = shape
    K = spec.kcut
    kr = np.arange(-K, K + 1)

    def basis(n):
        return np.exp(2j * np.pi * np.outer(kr, np.arange(n)) / n)   # (2K+1, n)

    ex, ey, ez = basis(nx), basis(ny), basis(nz)
    out = np.empty((3, nz, ny, nx), dtype)
    for comp in range(3):
        cube = _dense_cube(spec, comp)                       # [kx, ky, kz]
        t1 = cube.reshape(-1, 2 * K + 1) @ ez                # [kx*ky, z]
        t1 = t1.reshape(2 * K + 1, 2 * K + 1, nz)            # [kx, ky, z]
        t2 = t1.transpose(0, 2, 1) @ ey                      # [kx, z, y]
        t2 = np.ascontiguousarray(t2.transpose(1, 2, 0))     # [z, y, kx]
        for z0 in range(0, nz, zchunk):
            z1 = min(nz, z0 + zchunk)
            blk = t2[z0:z1].reshape(-1, 2 * K + 1) @ ex      # [(z,y), x]
            out[comp, z0:z1] = blk.real.reshape(z1 - z0, ny, nx)
    return out


def hit_field_at(spec: HitSpectrum, shape, points) -> np.ndarray:
    """Evaluate the field at points (P, 3) given as (x, y, z) coordinates.

    Direct sum over all wave vectors; for sampled checks of large grids.
    Returns (P, 3) float64.
    """
    L = np.asarray(shape, np.float64)
    pts = np.asarray(points, np.float64)
    out = np.empty((pts.shape[0], 3))
    kf = spec.k.astype(np.float64) / L[None, :]
    for s in range(0, pts.shape[0], 256):
        ph = np.exp(2j * np.pi * (pts[s:s + 256] @ kf.T))   # (p, M)
        out[s:s + 256] = (ph @ spec.b).real
    return out


def pipe_initial_velocity(shape, radius: float, centre, u_centre: float,
                          perturb: float, seed: int) -> np.ndarray:
    """Parabolic axial (z) profile u_z = u_c (1 - r^2/R^2) for r < R, zero
    outside, plus iid uniform perturbations in [-perturb*u_c, perturb*u_c] on
    every component of every node with r < R. Returns u[3, nz, ny, nx]."""
    nx, ny, nz = shape
    x = np.arange(nx, dtype=np.float64) - centre[0]
    y = np.arange(ny, dtype=np.float64) - centre[1]
    r2 = (y[:, None] ** 2 + x[None, :] ** 2)                  # [y, x]
    inside = r2 < radius * radius
    u = np.zeros((3, nz, ny, nx))
    u[2] = np.where(inside, u_centre * (1.0 - r2 / (radius * radius)), 0.0)[None]
    rng = np.random.default_rng(seed)
    noise = rng.uniform(-1.0, 1.0, size=(3, nz, ny, nx)) * (perturb * u_centre)
    u += noise * inside[None, None]
    return u


def random_velocity(shape, amp: float, seed: int) -> np.ndarray:
    """iid uniform components in [-amp, amp]; shape (nx, ny, nz) ->
    u[3, nz, ny, nx]."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(3, nz, ny, nx))


def random_density(shape, amp: float, seed: int) -> np.ndarray:
    """1 + iid uniform in [-amp, amp]; shape (nx, ny, nz) -> [nz, ny, nx]."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    return 1.0 + rng.uniform(-amp, amp, size=(nz, ny, nx))
