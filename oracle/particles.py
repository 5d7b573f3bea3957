"""Rigid spheres: state, motion and soft-sphere normal contact (FP64).

Equations of motion (Sec. 3.1 says only that the particle motion is updated
from the hydrodynamic force and torque; reading): with m = rho_p 4/3 pi r^3
and I = 2/5 m r^2, one explicit step of length 1
    U' = U + (F_h + F_c) / m,   X' = X + (U + U') / 2,   Omega' = Omega + T / I,
X' wrapped back into the periodic box with one explicit branch per axis.

Soft-sphere contact (Sec. 3.1: normal force only, no tangential friction,
no lubrication model): for an overlap delta = r_i + r_j - |X_i - X_j| > 0,
    F_i = (k_n delta - eta_n (U_i - U_j) . n) n,   n = (X_i - X_j)/|X_i - X_j|,
    k_n = m_eff (pi^2 + ln^2 e) / T_c^2,   eta_n = -2 m_eff ln e / T_c,
the linear spring-dashpot whose isolated head-on collision lasts T_c and
restitutes the normal speed by e. The paper does not give e or T_c;
defaults e = 0.97, T_c = 8 steps are readings.
"""
from dataclasses import dataclass

import numpy as np

from .geometry import min_image


@dataclass
class Particles:
    X: np.ndarray           # (np, 3) centres
    U: np.ndarray           # (np, 3) velocities
    Om: np.ndarray          # (np, 3) angular velocities
    r: np.ndarray           # (np,) radii
    rho: np.ndarray         # (np,) densities
    motion: str = "free"    # "free": equations of motion; "fixed": held in
                            # place; "prescribed": X advances by U, U and
                            # Omega held (forces are evaluated in every mode)

    @property
    def n(self):
        return len(self.r)

    @property
    def mass(self):
        return self.rho * (4.0 / 3.0) * np.pi * self.r ** 3

    @property
    def inertia(self):
        return 0.4 * self.mass * self.r ** 2

    def copy(self):
        return Particles(self.X.copy(), self.U.copy(), self.Om.copy(), self.r.copy(), self.rho.copy(), self.motion)


def contact_forces(P: Particles, shape, e: float, tc: float):
    L = np.asarray(shape, np.float64)
    F = np.zeros((P.n, 3))
    m = P.mass
    lne = np.log(e)
    for i in range(P.n):
        for j in range(P.n):
            if i == j:
                continue
            d = np.array([min_image(P.X[i, k] - P.X[j, k], L[k]) for k in range(3)])
            dist = np.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
            delta = P.r[i] + P.r[j] - dist
            if delta <= 0.0:
                continue
            n = d / dist
            meff = m[i] * m[j] / (m[i] + m[j])
            kn = meff * (np.pi ** 2 + lne * lne) / (tc * tc)
            eta = -2.0 * meff * lne / tc
            vn = (P.U[i] - P.U[j]) @ n
            F[i] += (kn * delta - eta * vn) * n
    return F


def wrap_position(x, L):
    x = np.where(x >= L, x - L, x)
    return np.where(x < 0.0, x + L, x)


def advance(P: Particles, F, T, shape):
    """One explicit step of the equations of motion; returns a new state."""
    if P.motion == "fixed":
        return P.copy()
    L = np.asarray(shape, np.float64)
    if P.motion == "prescribed":
        U1 = P.U.copy()
        Om1 = P.Om.copy()
    else:
        m = P.mass[:, None]
        I = P.inertia[:, None]
        U1 = P.U + F / m
        Om1 = P.Om + T / I
    X1 = P.X + 0.5 * (P.U + U1)
    X1 = np.stack([wrap_position(X1[:, k], L[k]) for k in range(3)], -1)
    return Particles(X1, U1, Om1, P.r.copy(), P.rho.copy(), P.motion)
