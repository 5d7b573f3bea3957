"""D3Q19 lattice and the d'Humieres multiple-relaxation-time moment basis.

The paper runs its particle-laden case on a D3Q19 MRT model following
d'Humieres et al. 2002 (Sec. 3.1). The velocity set, weights and the 19
moment polynomials below are the standard published ones; the basis is
written from its polynomial definitions, not typed as a matrix.

Velocity order used by the oracle: rest, the six faces, then the twelve
edges. Any order works; the HIP library uses its own table.
"""
import numpy as np

CS2 = 1.0 / 3.0

C = np.array([[0, 0, 0],
              [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
              [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
              [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int64)
Q = C.shape[0]
CF = C.astype(np.float64)
_C2 = (CF * CF).sum(1)
W = np.where(_C2 == 0, 1.0 / 3.0, np.where(_C2 == 1, 1.0 / 18.0, 1.0 / 36.0))
OPP = np.array([int(np.flatnonzero((C == -C[i]).all(1))[0]) for i in range(Q)])


def moment_basis() -> np.ndarray:
    """Rows of M as polynomials of the discrete velocity c (d'Humieres 2002):
    rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx, p_ww, pi_ww,
    p_xy, p_yz, p_xz, m_x, m_y, m_z."""
    cx, cy, cz = CF.T
    c2 = _C2
    rows = [
        np.ones(Q),
        19.0 * c2 - 30.0,
        (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0,
        cx, (5.0 * c2 - 9.0) * cx,
        cy, (5.0 * c2 - 9.0) * cy,
        cz, (5.0 * c2 - 9.0) * cz,
        3.0 * cx * cx - c2, (3.0 * c2 - 5.0) * (3.0 * cx * cx - c2),
        cy * cy - cz * cz, (3.0 * c2 - 5.0) * (cy * cy - cz * cz),
        cx * cy, cy * cz, cx * cz,
        (cy * cy - cz * cz) * cx, (cz * cz - cx * cx) * cy, (cx * cx - cy * cy) * cz,
    ]
    return np.array(rows)


M = moment_basis()
M_INV = np.linalg.inv(M)

# Moment groups (row indices of M).
ROW_RHO, ROW_E, ROW_EPS = 0, 1, 2
ROWS_J = (3, 5, 7)
ROWS_Q = (4, 6, 8)
ROWS_NU = (9, 11, 13, 14, 15)     # the five stress moments: shear viscosity
ROWS_PI = (10, 12)
ROWS_M = (16, 17, 18)

# d'Humieres 2002 relaxation rates for the non-hydrodynamic moments. The
# paper names the model but not the values; these are the usual ones.
DEFAULT_RATES = dict(s_e=1.19, s_eps=1.4, s_q=1.2, s_pi=1.4, s_m=1.98)


def relaxation_vector(tau: float, s_e: float, s_eps: float, s_q: float,
                      s_pi: float, s_m: float) -> np.ndarray:
    """Diagonal of S. Conserved moments (rho, j) get rate 0; the stress
    moments relax with 1/tau, so the kinematic viscosity is (tau - 1/2)/3."""
    s = np.zeros(Q)
    s[ROW_E] = s_e
    s[ROW_EPS] = s_eps
    for r in ROWS_Q:
        s[r] = s_q
    for r in ROWS_NU:
        s[r] = 1.0 / tau
    for r in ROWS_PI:
        s[r] = s_pi
    for r in ROWS_M:
        s[r] = s_m
    return s


def viscosity(tau: float) -> float:
    return (tau - 0.5) * CS2
