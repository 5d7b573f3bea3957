"""Equilibrium, Guo forcing, MRT collision and pull streaming (FP64).

* Equilibrium: the compressible second-order polynomial
  f_i^eq = w_i rho [1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u]; its moments define
  m^eq = M f^eq. The paper does not say which form it used; this is the
  reading.
* Forcing: the paper drives the pipe by a body force rho*g (Sec. 2.1) and the
  immersed boundary adds a force density (Sec. 2.1, Sec. 3.1) but names no
  forcing scheme. Reading: Guo et al. in MRT form,
      m~ = m - S (m - m^eq) + (I - S/2) M Fbar,
      Fbar_i = w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F,
  with the half-force velocity u = (sum_i c_i f_i + F/2) / rho.
* Collision in moment space with the d'Humieres basis (Sec. 3.1); f~ = M^-1 m~.
* Streaming, pull form: f_i(x, t+1) = f~_i(x - c_i, t) on a periodic box.

Population arrays are (19, nz, ny, nx); vectors are (3, nz, ny, nx) or any
shape broadcastable against it.
"""
import numpy as np

from .lattice import C, CF, M, M_INV, Q, W


def _bw(a, ndim):
    """Reshape a length-19 table to broadcast against (19, *spatial)."""
    return a.reshape((-1,) + (1,) * ndim)


def equilibrium(rho, u):
    """f^eq(rho, u); rho (*s), u (3, *s) -> (19, *s)."""
    rho = np.asarray(rho, np.float64)
    u = np.asarray(u, np.float64)
    nd = u.ndim - 1
    cu = np.tensordot(CF, u, axes=(1, 0))
    usq = (u * u).sum(0)
    return _bw(W, nd) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq)


def guo_source(u, F):
    """Fbar_i = w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F  -> (19, *s)."""
    u = np.asarray(u, np.float64)
    F = np.broadcast_to(np.asarray(F, np.float64), u.shape)
    nd = u.ndim - 1
    cu = np.tensordot(CF, u, axes=(1, 0))
    cF = np.tensordot(CF, F, axes=(1, 0))
    uF = (u * F).sum(0)
    return _bw(W, nd) * (3.0 * (cF - uF) + 9.0 * cu * cF)


def density(f):
    return f.sum(0)


def momentum(f):
    """sum_i c_i f_i -> (3, *s)."""
    return np.tensordot(CF.T, f, axes=(1, 0))


def velocity(f, F):
    """Half-force velocity u = (sum_i c_i f_i + F/2) / rho."""
    rho = density(f)
    F = np.broadcast_to(np.asarray(F, np.float64), (3,) + rho.shape)
    return (momentum(f) + 0.5 * F) / rho


def collide(f, F, s):
    """MRT + Guo collision of pre-collision populations f (19, *s) under the
    total force density F (3, *s) with relaxation diagonal s (19,).

    Returns (f_post, rho, u) where u is the half-force velocity used in the
    collision."""
    shape = f.shape[1:]
    rho = density(f)
    u = velocity(f, F)
    Fb = np.broadcast_to(np.asarray(F, np.float64), (3,) + shape)
    m = M @ f.reshape(Q, -1)
    meq = M @ equilibrium(rho, u).reshape(Q, -1)
    mF = M @ guo_source(u, Fb).reshape(Q, -1)
    s = s[:, None]
    mpost = m - s * (m - meq) + (1.0 - 0.5 * s) * mF
    return (M_INV @ mpost).reshape(f.shape), rho, u


def stream_pull(ft):
    """f_i(x) = ft_i(x - c_i), periodic in all three directions."""
    f = np.empty_like(ft)
    for i in range(Q):
        f[i] = np.roll(ft[i], shift=(C[i, 2], C[i, 1], C[i, 0]), axis=(0, 1, 2))
    return f


def neighbour(idx_zyx, i, shape_zyx, k=1):
    """Periodic index of x + k c_i for integer (z, y, x) tuples."""
    z, y, x = idx_zyx
    nz, ny, nx = shape_zyx
    return ((z + k * C[i, 2]) % nz, (y + k * C[i, 1]) % ny, (x + k * C[i, 0]) % nx)
