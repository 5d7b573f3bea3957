"""Refilling of nodes a moving particle uncovers (Sec. 3.1; FP64).

The paper uses Caiazzo's scheme without giving its formula. Reading taken
here: velocity-constrained extrapolation along the lattice direction
closest to the outward normal.

For a node x uncovered by particle p (solid at step n, fluid at n+1):
 1. d = x - X_p (minimum image, new particle position). c_k = the lattice
    direction maximising c_k . d; ties go to the lexicographically largest
    (c_x, c_y, c_z).
 2. "Valid" neighbours are fluid both before and after the move (so they
    hold post-collision populations of step n+1). Extrapolate
       f_ext = 3 f(x+c_k) - 3 f(x+2c_k) + f(x+3c_k)   if all three are valid,
       f_ext = 2 f(x+c_k) - f(x+2c_k)                  else if both are,
    else f_ext = f_eq(rho_avg, u_avg) from the valid nearest neighbours
    (mean density and mean raw velocity sum_i c_i f_i / rho), else
    f_eq(1, u_w).
 3. Replace the equilibrium part by the wall velocity:
       f = f_ext - f_eq(rho_ext, u_ext) + f_eq(rho_ext, u_w),
    rho_ext = sum f_ext, u_ext = sum c f_ext / rho_ext,
    u_w = U_p + Omega_p x d.
The momentum sum_i c_i f_i of each refilled node is taken from its particle
(added with a minus sign to the particle force of the next step); the
momentum of a node a particle covers is given to it (reading).
"""
import numpy as np

from .collide import equilibrium
from .geometry import _offsets_many
from .lattice import C, CF, Q


def extrapolation_direction(d):
    """Index (oracle order) of the direction maximising c . d."""
    best = None
    for k in range(1, Q):
        v = (CF[k, 0] * d[0] + CF[k, 1] * d[1]) + CF[k, 2] * d[2]
        key = (v, C[k, 0], C[k, 1], C[k, 2])
        if best is None or key > best[0]:
            best = (key, k)
    return best[1]


def refill_node(ft, valid, xyz, p, P, shape):
    """Populations (19,) for uncovered node xyz of particle p."""
    nx, ny, nz = shape
    x, y, z = xyz
    d = _offsets_many(P.X, np.array([p]), np.array([xyz]), shape)[0]
    uw = P.U[p] + np.cross(P.Om[p], d)
    k = extrapolation_direction(d)

    def node(s):
        return ((x + s * C[k, 0]) % nx, (y + s * C[k, 1]) % ny, (z + s * C[k, 2]) % nz)

    def ok(s):
        xx, yy, zz = node(s)
        return bool(valid[zz, yy, xx])

    def f_at(s):
        xx, yy, zz = node(s)
        return ft[:, zz, yy, xx]

    if ok(1) and ok(2) and ok(3):
        fext = 3.0 * f_at(1) - 3.0 * f_at(2) + f_at(3)
    elif ok(1) and ok(2):
        fext = 2.0 * f_at(1) - f_at(2)
    else:
        rhos, us = [], []
        for i in range(1, Q):
            xx, yy, zz = (x + C[i, 0]) % nx, (y + C[i, 1]) % ny, (z + C[i, 2]) % nz
            if valid[zz, yy, xx]:
                f = ft[:, zz, yy, xx]
                rho = f.sum()
                rhos.append(rho)
                us.append(CF.T @ f / rho)
        if rhos:
            fext = equilibrium(np.mean(rhos), np.mean(us, axis=0))
        else:
            fext = equilibrium(1.0, uw)
    rho_e = fext.sum()
    u_e = CF.T @ fext / rho_e
    return fext - equilibrium(rho_e, u_e) + equilibrium(rho_e, uw)
