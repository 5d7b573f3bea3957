"""Interpolated bounce-back and the Galilean-invariant momentum exchange
(Sec. 3.1, Sec. 2.1; FP64).

For a link from fluid node x_f in direction a (towards the solid) with wall
fraction q, the population entering x_f from the wall, direction abar, is
interpolated from post-collision values f~ at time t (Bouzidi, Firdaouss &
Lallemand 2001), plus the moving-wall term delta = -6 w_a (c_a . u_w)
(reference density 1):

  quadratic, q < 1/2:  q(1+2q) f~_a(x_f) + (1-4q^2) f~_a(x_f-c_a)
                       - q(1-2q) f~_a(x_f-2c_a) + delta
  quadratic, q >= 1/2: f~_a(x_f)/(q(2q+1)) + (2q-1)/q f~_abar(x_f)
                       - (2q-1)/(2q+1) f~_abar(x_f-c_a) + delta/(q(2q+1))
  linear, q < 1/2:     2q f~_a(x_f) + (1-2q) f~_a(x_f-c_a) + delta
  linear, q >= 1/2:    f~_a(x_f)/(2q) + (2q-1)/(2q) f~_abar(x_f) + delta/(2q)
  single node:         f~_a(x_f) + delta   (halfway bounce-back; stands in
                       for the Zhao & Yong scheme the paper cites, whose
                       formula is not reproduced here)

u_w is the rigid-body velocity U + Omega x (x_w - X) at the wall point
x_w = x_f + q c_a. Force on the solid from one link (Wen et al. 2014):
  F = (c_a - u_w) f~_a(x_f) - (c_abar - u_w) f_abar(x_f, t+1),
torque (x_w - X) x F (lever arm at x_w: reading).
"""
import numpy as np

from .geometry import SCHEME_HALFWAY, SCHEME_LINEAR, SCHEME_QUADRATIC, _offsets_many
from .lattice import C, CF, OPP, W


def wall_velocity(links, X, U, Om, shape):
    """u_w at every link's wall point and the lever arm x_w - X (zero for the
    static wall)."""
    p = links["p"]
    n = len(p)
    uw = np.zeros((n, 3))
    arm = np.zeros((n, 3))
    sph = p >= 0
    if sph.any():
        d = _offsets_many(X, p[sph], links["xf"][sph], shape)
        arm_s = d + links["q"][sph, None] * CF[links["a"][sph]]
        uw[sph] = U[p[sph]] + np.cross(Om[p[sph]], arm_s)
        arm[sph] = arm_s
    return uw, arm


def _at(ft, a, xyz, shape):
    nx, ny, nz = shape
    return ft[a, xyz[:, 2] % nz, xyz[:, 1] % ny, xyz[:, 0] % nx]


def bounce_values(ft, links, uw, shape):
    """f_abar(x_f, t+1) for every link."""
    a = links["a"]
    ab = OPP[a]
    q = links["q"]
    xf = links["xf"]
    c = C[a]
    fa0 = _at(ft, a, xf, shape)
    fa1 = _at(ft, a, xf - c, shape)
    fa2 = _at(ft, a, xf - 2 * c, shape)
    fb0 = _at(ft, ab, xf, shape)
    fb1 = _at(ft, ab, xf - c, shape)
    delta = -6.0 * W[a] * (CF[a] * uw).sum(1)
    with np.errstate(invalid="ignore", divide="ignore"):   # unselected branches may divide by q = 0
        quad_lo = q * (1 + 2 * q) * fa0 + (1 - 4 * q * q) * fa1 - q * (1 - 2 * q) * fa2 + delta
        quad_hi = (fa0 / (q * (2 * q + 1)) + (2 * q - 1) / q * fb0 - (2 * q - 1) / (2 * q + 1) * fb1
                   + delta / (q * (2 * q + 1)))
        lin_lo = 2 * q * fa0 + (1 - 2 * q) * fa1 + delta
        lin_hi = fa0 / (2 * q) + (2 * q - 1) / (2 * q) * fb0 + delta / (2 * q)
    half = fa0 + delta
    lo = q < 0.5
    s = links["scheme"]
    return np.where(s == SCHEME_QUADRATIC, np.where(lo, quad_lo, quad_hi),
                    np.where(s == SCHEME_LINEAR, np.where(lo, lin_lo, lin_hi), half))


def link_forces(ft, fb, links, uw, arm, shape):
    """GIMEM force and torque of every link on its solid."""
    a = links["a"]
    fa0 = _at(ft, a, links["xf"], shape)
    ca = CF[a]
    F = (ca - uw) * fa0[:, None] + (ca + uw) * fb[:, None]
    T = np.cross(arm, F)
    return F, T
