"""D3Q27 lattice for the turbulent pipe (Sec. 2.2), FP64.

Test infrastructure: only the tests and the smoke check use this module.

The paper's pipe runs use a D3Q27 multiple-relaxation-time model driven with
one relaxation parameter for all moments, so that the bulk viscosity equals
the shear viscosity, and name (without activating it) the option of a longer
relaxation time for the energy mode to damp acoustic noise (Sec. 2.2, the
discussion of the pressure term E_Pr). It gives no basis, equilibrium or
forcing. Readings this oracle fixes:

* Velocities: the 27 vectors of {-1, 0, 1}^3; weights are products of the
  D1Q3 weights 2/3 (c = 0) and 1/6 (c = +-1): 8/27, 2/27, 1/54, 1/216 for
  |c|^2 = 0, 1, 2, 3; c_s^2 = 1/3.
* Moment basis: products phi_a(c_x) phi_b(c_y) phi_c(c_z) of the D1Q3
  polynomials 1, c, 3c^2 - 1, which are orthogonal under those weights,
  except that the three products with one factor 3c^2 - 1 and two factors
  1 are recombined into the energy mode |c|^2 - 1 (their sum over 3) and two
  traceless combinations; the recombination is orthogonal, so the basis stays
  orthogonal.
* Collision in moment space, m~ = m - S (m - m_eq) + (I - S/2) M Fbar, with
  S = 1/tau on every non-conserved moment except the energy mode, which
  relaxes at 1/tau_bulk. tau_bulk = tau is the paper's single relaxation
  parameter, and then the collision is BGK. Shear viscosity
  nu = (tau - 1/2)/3; the energy mode's nu_b = (tau_bulk - 1/2)/3, equal to
  nu at one parameter; the bulk viscosity of the Navier-Stokes stress is
  zeta = 2 rho nu_b / 3.
* Equilibrium: the second-order polynomial
  w_i rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u]; forcing: Guo et al.,
  Fbar_i = w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F with the half-force velocity
  u = (sum_i c_i f_i + F/2) / rho (the same readings as the D3Q19 model).
* Pipe wall: the links and the linear interpolated bounce-back of the pipe
  (Sec. 2.1: the pipe is run with the linear scheme), over the 26 moving
  directions; the wall is static. Step order: pull streaming with the
  bounce-back values at the links, then collision with the body force at the
  fluid nodes.

Population arrays are (27, nz, ny, nx).
"""
import itertools

import numpy as np

from .geometry import SCHEME_HALFWAY, SCHEME_LINEAR, pipe_q, pipe_solid

CS2 = 1.0 / 3.0

C = np.array(list(itertools.product((0, 1, -1), repeat=3)), dtype=np.int64)[:, ::-1].copy()  # rows (cx, cy, cz)
Q = C.shape[0]
CF = C.astype(np.float64)
_W1 = {0: 2.0 / 3.0, 1: 1.0 / 6.0, -1: 1.0 / 6.0}
W = np.array([_W1[int(a)] * _W1[int(b)] * _W1[int(c)] for a, b, c in C])
OPP = np.array([int(np.flatnonzero((C == -C[i]).all(1))[0]) for i in range(Q)])


def _p1(k, c):
    """D1Q3 orthogonal polynomial of degree k at c."""
    return (np.ones_like(c), c, 3.0 * c * c - 1.0)[k]


def moment_basis():
    """(27, 27) basis rows and the row index of the energy mode. The rows
    with degrees (2,0,0), (0,2,0), (0,0,2) are replaced by their sum / 3
    (= |c|^2 - 1, the energy mode) and by the traceless (2,0,0) - (0,2,0)
    and (2,0,0) + (0,2,0) - 2 (0,0,2)."""
    rows, e_row = [], None
    cx, cy, cz = CF.T
    deg = list(itertools.product(range(3), repeat=3))
    pure2 = {(2, 0, 0), (0, 2, 0), (0, 0, 2)}
    for a, b, c in deg:
        if (a, b, c) in pure2:
            continue
        rows.append(_p1(a, cx) * _p1(b, cy) * _p1(c, cz))
    px, py, pz = _p1(2, cx), _p1(2, cy), _p1(2, cz)
    e_row = len(rows)
    rows.append((px + py + pz) / 3.0)
    rows.append(px - py)
    rows.append(px + py - 2.0 * pz)
    return np.array(rows), e_row


M, ROW_E = moment_basis()
M_INV = np.linalg.inv(M)
ROW_RHO = 0
ROWS_J = tuple(int(np.flatnonzero(np.all(np.isclose(M, CF[:, k][None, :]), axis=1))[0]) for k in range(3))


def relaxation_vector(tau, tau_bulk=None):
    s = np.full(Q, 1.0 / tau)
    s[ROW_E] = 1.0 / (tau if tau_bulk is None or tau_bulk == 0 else tau_bulk)
    s[ROW_RHO] = 0.0
    for r in ROWS_J:
        s[r] = 0.0
    return s


def _bw(a, nd):
    return a.reshape((-1,) + (1,) * nd)


def equilibrium(rho, u):
    rho = np.asarray(rho, np.float64)
    u = np.asarray(u, np.float64)
    nd = u.ndim - 1
    cu = np.tensordot(CF, u, axes=(1, 0))
    usq = (u * u).sum(0)
    return _bw(W, nd) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq)


def guo_source(u, F):
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
    return np.tensordot(CF.T, f, axes=(1, 0))


def collide(f, F, s):
    """Moment-space collision of f (27, *s) under force density F (3, *s);
    returns (f~, rho, u) with u the half-force velocity."""
    shape = f.shape[1:]
    rho = density(f)
    Fb = np.broadcast_to(np.asarray(F, np.float64), (3,) + shape)
    u = (momentum(f) + 0.5 * Fb) / rho
    m = M @ f.reshape(Q, -1)
    meq = M @ equilibrium(rho, u).reshape(Q, -1)
    mF = M @ guo_source(u, Fb).reshape(Q, -1)
    s = np.asarray(s)[:, None]
    mpost = m - s * (m - meq) + (1.0 - 0.5 * s) * mF
    return (M_INV @ mpost).reshape(f.shape), rho, u


def stream_pull(ft):
    f = np.empty_like(ft)
    for i in range(Q):
        f[i] = np.roll(ft[i], shift=(C[i, 2], C[i, 1], C[i, 0]), axis=(0, 1, 2))
    return f


def pipe_links(shape, R, cx, cy):
    """Links of the fluid nodes (r^2 < R^2 about (cx, cy)) towards the wall,
    over the 26 moving directions: xf (L, 3), a (L,), q (L,), scheme (L,).
    The linear scheme needs x_f - c_a fluid when q < 1/2, else the link falls
    back to halfway bounce-back."""
    solid = pipe_solid(shape, R, cx, cy)
    fluid = ~solid
    nx, ny, nz = shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = {k: [] for k in ("xf", "a", "q", "scheme")}
    for a in range(Q):
        if not C[a].any():
            continue
        ccx, ccy, ccz = C[a]
        hit = fluid & np.roll(solid, shift=(-ccz, -ccy, -ccx), axis=(0, 1, 2))
        if not hit.any():
            continue
        xf = np.stack([xx[hit], yy[hit], zz[hit]], -1)
        dxy = np.stack([xf[:, 0] - cx, xf[:, 1] - cy], -1).astype(np.float64)
        q = pipe_q(dxy, np.broadcast_to(CF[a, :2], dxy.shape), R)
        f1 = np.roll(fluid, shift=(ccz, ccy, ccx), axis=(0, 1, 2))[hit]
        scheme = np.where((q >= 0.5) | f1, SCHEME_LINEAR, SCHEME_HALFWAY)
        out["xf"].append(xf)
        out["a"].append(np.full(len(q), a))
        out["q"].append(q)
        out["scheme"].append(scheme)
    return {k: np.concatenate(v) for k, v in out.items()}, solid


def bounce_linear(ft, links, shape):
    """f_abar(x_f, t+1) at every static-wall link from post-collision f~."""
    nx, ny, nz = shape
    a, q, xf = links["a"], links["q"], links["xf"]
    ab = OPP[a]

    def at(i, p):
        return ft[i, p[:, 2] % nz, p[:, 1] % ny, p[:, 0] % nx]

    fa0 = at(a, xf)
    fa1 = at(a, xf - C[a])
    fb0 = at(ab, xf)
    with np.errstate(invalid="ignore", divide="ignore"):
        lo = 2.0 * q * fa0 + (1.0 - 2.0 * q) * fa1
        hi = fa0 / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * fb0
    lin = np.where(q < 0.5, lo, hi)
    return np.where(links["scheme"] == SCHEME_LINEAR, lin, fa0)


class Sim27:
    """FP64 reference run of the D3Q27 solver: periodic box, or a pipe along
    z with the linear interpolated bounce-back wall."""

    def __init__(self, shape, tau, tau_bulk=0.0, body_force=(0.0, 0.0, 0.0), pipe=None):
        self.shape = tuple(shape)
        nx, ny, nz = shape
        self.zyx = (nz, ny, nx)
        self.s = relaxation_vector(tau, tau_bulk)
        self.F = np.broadcast_to(np.asarray(body_force, np.float64).reshape(3, 1, 1, 1), (3,) + self.zyx).copy()
        self.links, self.solid = (None, np.zeros(self.zyx, bool))
        if pipe is not None:
            self.links, self.solid = pipe_links(self.shape, *pipe)
            self.F[:, self.solid] = 0.0
        self.set_fields(np.zeros((3,) + self.zyx))

    def set_fields(self, u, rho=None):
        u = np.asarray(u, np.float64).reshape((3,) + self.zyx)
        rho = np.ones(self.zyx) if rho is None else np.asarray(rho, np.float64).reshape(self.zyx)
        self.ft = equilibrium(rho, u)
        self.ft[:, self.solid] = np.nan
        self.rho, self.u = rho.copy(), u.copy()
        self.steps = 0

    def step(self, n=1):
        for _ in range(n):
            f = stream_pull(self.ft)
            if self.links is not None and len(self.links["a"]):
                L = self.links
                f[OPP[L["a"]], L["xf"][:, 2], L["xf"][:, 1], L["xf"][:, 0]] = bounce_linear(self.ft, L, self.shape)
            f[:, self.solid] = 0.0
            f[0, self.solid] = 1.0
            self.ft, rho, u = collide(f, self.F, self.s)
            self.ft[:, self.solid] = np.nan
            rho[self.solid] = np.nan
            u[:, self.solid] = np.nan
            self.rho, self.u = rho, u
            self.steps += 1
        return self
