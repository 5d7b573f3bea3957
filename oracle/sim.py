"""Time-stepping driver of the FP64 oracle.

The paper gives no step order (it cites each scheme); the order below is the
reading this oracle fixes, and the HIP library follows it.

State at integer step n: post-collision populations f~(x, n) (NaN at nodes
inside interpolated-bounce-back solids, so any read of them shows up),
the particle state (X, U, Omega) in FP64 and the momentum handed over by
covered/uncovered nodes at the end of step n-1.

Interpolated bounce-back, step n -> n+1 (Sec. 3.1):
  1. geometry at X^n: owner map, boundary links, q, fallback scheme
  2. pull streaming; at every link the entering population comes from the
     interpolated bounce-back formula instead of the solid node
  3. link forces (GIMEM) summed per particle
  4. MRT + Guo collision at fluid nodes (body force on fluid nodes only)
  5. contact forces from X^n, U^n; equations of motion -> X^{n+1}
  6. geometry at X^{n+1}; nodes that became fluid are refilled, their
     momentum taken from the particle; nodes that became solid give their
     momentum to it; both enter the force of the next step.
Immersed boundary, step n -> n+1 (Sec. 2.1, Sec. 3.1):
  1. pull streaming at every node (the interior holds virtual fluid)
  2. rho and u* = (sum c f + F_body/2)/rho
  3. markers at X^n, desired velocity U^n + Omega^n x (X_l - X^n)
  4. multi-direct forcing: 1 + ibm_iters passes
  5. collision with F_body + f_IB
  6. particle force -sum F_l dV_l plus the change of the Kempe inner
     momentum sum alpha u (Sec. 3.1), contact forces, equations of motion.
The macroscopic fields of step n+1 are the density and half-force velocity
used in that step's collision.
"""
from dataclasses import dataclass, field

import numpy as np

from . import collide as col
from . import geometry as geo
from . import ibb, ibm, refill
from .lattice import CF, OPP, DEFAULT_RATES, relaxation_vector
from .particles import Particles, advance, contact_forces

# set_particles modes
SET_STATE, RELEASE, SET_RIGID = 0, 1, 2


@dataclass
class Config:
    shape: tuple = (32, 32, 32)          # (nx, ny, nz)
    tau: float = 0.6
    s_e: float = DEFAULT_RATES["s_e"]
    s_eps: float = DEFAULT_RATES["s_eps"]
    s_q: float = DEFAULT_RATES["s_q"]
    s_pi: float = DEFAULT_RATES["s_pi"]
    s_m: float = DEFAULT_RATES["s_m"]
    body_force: tuple = (0.0, 0.0, 0.0)
    bc: str = "none"                     # "none" | "ibb" | "ibm"
    ibb_max_order: int = 2
    ibm_retraction: float = 0.0
    ibm_iters: int = 2
    wall: str = "none"                   # "none" | "pipe_z"
    pipe_radius: float = 0.0
    pipe_cx: float = 0.0
    pipe_cy: float = 0.0
    coll_restitution: float = 0.97
    coll_tc_steps: float = 8.0

    @property
    def zyx(self):
        nx, ny, nz = self.shape
        return (nz, ny, nx)

    def rates(self):
        return relaxation_vector(self.tau, self.s_e, self.s_eps, self.s_q, self.s_pi, self.s_m)


@dataclass
class State:
    ft: np.ndarray                        # (19, nz, ny, nx) post-collision
    rho: np.ndarray                       # (nz, ny, nx) of the last collision
    u: np.ndarray                         # (3, nz, ny, nx)
    step: int = 0
    P: Particles = None
    owner: np.ndarray = None              # geometry of the current step (IBB)
    links: dict = None
    F_rc: np.ndarray = None               # cover/uncover momentum for the next step
    T_rc: np.ndarray = None
    Iu: np.ndarray = None                 # Kempe inner momentum (IBM)
    IL: np.ndarray = None
    F_h: np.ndarray = None                # hydrodynamic force/torque of the last step
    T_h: np.ndarray = None
    F_c: np.ndarray = None                # contact force of the last step
    F_l: np.ndarray = None                # marker forces of the last step (IBM)
    extra: dict = field(default_factory=dict)


class Sim:
    """Plain FP64 reference run of the method."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        self.s = cfg.rates()
        zyx = cfg.zyx
        self.wall_solid = None
        if cfg.wall == "pipe_z":
            self.wall_solid = geo.pipe_solid(cfg.shape, cfg.pipe_radius, cfg.pipe_cx, cfg.pipe_cy)
        self.F_body = np.broadcast_to(np.asarray(cfg.body_force, np.float64).reshape(3, 1, 1, 1),
                                      (3,) + zyx).copy()
        if cfg.bc == "ibm" and self.wall_solid is not None:
            # The virtual fluid outside the pipe is not driven (reading).
            self.F_body[:, self.wall_solid] = 0.0
        rho = np.ones(zyx)
        u = np.zeros((3,) + zyx)
        self.state = State(ft=col.equilibrium(rho, u), rho=rho, u=u)
        self._empty_particles()

    # -- helpers ----------------------------------------------------------
    def _empty_particles(self):
        st = self.state
        st.P = Particles(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros(0))
        self._refresh_geometry()
        z = np.zeros((0, 3))
        st.F_rc, st.T_rc, st.Iu, st.IL, st.F_h, st.T_h, st.F_c = z, z, z, z, z, z, z

    def _refresh_geometry(self):
        st = self.state
        if self.cfg.bc == "ibb":
            st.owner = geo.owner_map(self.cfg.shape, st.P.X, st.P.r, self.wall_solid)
            pipe = (self.cfg.pipe_radius, self.cfg.pipe_cx, self.cfg.pipe_cy) if self.wall_solid is not None else None
            st.links = geo.build_links(st.owner, st.P.X, st.P.r, self.cfg.shape, self.cfg.ibb_max_order, pipe)
            st.ft[:, st.owner != -1] = np.nan
        else:
            st.owner = None
            st.links = None

    def fluid_mask(self):
        if self.cfg.bc == "ibb":
            return self.state.owner == -1
        return np.ones(self.cfg.zyx, bool)

    # -- fields -----------------------------------------------------------
    def set_fields(self, u, rho=None):
        zyx = self.cfg.zyx
        u = np.asarray(u, np.float64).reshape((3,) + zyx)
        rho = np.ones(zyx) if rho is None else np.asarray(rho, np.float64).reshape(zyx)
        P = self.state.P
        self.state = State(ft=col.equilibrium(rho, u), rho=rho.copy(), u=u.copy())
        self.state.P = P
        self._refresh_geometry()
        n = P.n
        st = self.state
        st.F_rc, st.T_rc = np.zeros((n, 3)), np.zeros((n, 3))
        st.F_h, st.T_h, st.F_c = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3))
        if self.cfg.bc == "ibm":
            st.Iu, st.IL = ibm.inner_integrals(st.u, P.X, P.r, self.cfg.shape)

    def fields(self):
        return self.state.u, self.state.rho

    # -- particles --------------------------------------------------------
    def set_particles(self, X, U=None, Om=None, r=None, rho_p=None, mode=SET_STATE, motion="free"):
        """Places spheres. RELEASE (Sec. 3.1): U = fluid velocity averaged over
        the particle volume (Kempe-fraction weighted), Omega = 0, and the
        velocity inside the particle is overwritten once by the rigid-body
        motion (equilibrium at the local density). SET_RIGID: U and Omega as
        given, the interior overwritten once by U + Omega x (x - X)."""
        st = self.state
        X = np.atleast_2d(np.asarray(X, np.float64)).copy()
        n = len(X)
        U = np.zeros((n, 3)) if U is None else np.atleast_2d(np.asarray(U, np.float64)).copy()
        Om = np.zeros((n, 3)) if Om is None else np.atleast_2d(np.asarray(Om, np.float64)).copy()
        r = np.asarray(r, np.float64).reshape(n).copy()
        rho_p = np.ones(n) if rho_p is None else np.asarray(rho_p, np.float64).reshape(n).copy()
        shape = self.cfg.shape
        if mode == RELEASE:
            for p in range(n):
                nodes = geo.box_nodes(X[p], r[p] + 1.0, shape)
                alpha = ibm.solid_fraction(X[p], r[p], nodes, shape)
                uu = st.u[:, nodes[:, 2], nodes[:, 1], nodes[:, 0]]
                U[p] = (uu * alpha[None]).sum(1) / alpha.sum()
            Om[:] = 0.0
        if mode in (RELEASE, SET_RIGID):
            # interior: equilibrium of the local density and the rigid-body
            # velocity U + Omega x (x - X)
            inside = geo.owner_map(shape, X, r, None)
            for p in range(n):
                zz, yy, xx = np.nonzero(inside == p)
                rho = st.rho[zz, yy, xx]
                d = np.stack([geo.min_image(xx - X[p, 0], shape[0]), geo.min_image(yy - X[p, 1], shape[1]),
                              geo.min_image(zz - X[p, 2], shape[2])], -1)
                urig = (U[p][None, :] + np.cross(np.broadcast_to(Om[p], d.shape), d)).T
                st.ft[:, zz, yy, xx] = col.equilibrium(rho, urig)
                st.u[:, zz, yy, xx] = urig
        st.P = Particles(X, U, Om, r, rho_p, motion)
        self._refresh_geometry()
        st.F_rc, st.T_rc = np.zeros((n, 3)), np.zeros((n, 3))
        st.F_h, st.T_h, st.F_c = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3))
        if self.cfg.bc == "ibm":
            st.Iu, st.IL = ibm.inner_integrals(st.u, X, r, shape)

    def forces(self):
        st = self.state
        return st.F_h.copy(), st.T_h.copy(), st.F_c.copy()

    # -- stepping ---------------------------------------------------------
    def step(self, n: int = 1):
        for _ in range(n):
            if self.cfg.bc == "ibb":
                self._step_ibb()
            elif self.cfg.bc == "ibm":
                self._step_ibm()
            else:
                self._step_plain()

    def _step_plain(self):
        st = self.state
        f = col.stream_pull(st.ft)
        st.ft, st.rho, st.u = col.collide(f, self.F_body, self.s)
        st.step += 1

    def _contact(self):
        st = self.state
        if st.P.n == 0 or st.P.motion != "free":
            return np.zeros((st.P.n, 3))
        return contact_forces(st.P, self.cfg.shape, self.cfg.coll_restitution, self.cfg.coll_tc_steps)

    def _step_ibb(self):
        cfg, st = self.cfg, self.state
        shape = cfg.shape
        P = st.P
        links = st.links
        owner = st.owner
        f = col.stream_pull(st.ft)
        uw, arm = ibb.wall_velocity(links, P.X, P.U, P.Om, shape)
        fb = ibb.bounce_values(st.ft, links, uw, shape)
        xf = links["xf"]
        f[OPP[links["a"]], xf[:, 2], xf[:, 1], xf[:, 0]] = fb
        Fl, Tl = ibb.link_forces(st.ft, fb, links, uw, arm, shape)
        F_h = np.zeros((P.n, 3))
        T_h = np.zeros((P.n, 3))
        sph = links["p"] >= 0
        np.add.at(F_h, links["p"][sph], Fl[sph])
        np.add.at(T_h, links["p"][sph], Tl[sph])
        fluid = owner == -1
        F = self.F_body * fluid[None]
        ft_new, rho, u = col.collide(f, F, self.s)
        ft_new[:, ~fluid] = np.nan
        rho = np.where(fluid, rho, np.nan)
        u = np.where(fluid[None], u, np.nan)
        F_h += st.F_rc
        T_h += st.T_rc
        F_c = self._contact()
        P1 = advance(P, F_h + F_c, T_h, shape)
        # geometry at X^{n+1}: cover / uncover
        owner1 = geo.owner_map(shape, P1.X, P1.r, self.wall_solid)
        valid = fluid & (owner1 == -1)
        F_rc = np.zeros((P.n, 3))
        T_rc = np.zeros((P.n, 3))
        zz, yy, xx = np.nonzero(fluid & (owner1 >= 0))
        for z, y, x in zip(zz, yy, xx):
            p = owner1[z, y, x]
            mom = CF.T @ ft_new[:, z, y, x]
            d = geo._offsets_many(P1.X, np.array([p]), np.array([[x, y, z]]), shape)[0]
            F_rc[p] += mom
            T_rc[p] += np.cross(d, mom)
        zz, yy, xx = np.nonzero((owner >= 0) & (owner1 == -1))
        fills = []
        for z, y, x in zip(zz, yy, xx):
            p = owner[z, y, x]
            fr = refill.refill_node(ft_new, valid, (x, y, z), p, P1, shape)
            fills.append((z, y, x, fr))
            mom = CF.T @ fr
            d = geo._offsets_many(P1.X, np.array([p]), np.array([[x, y, z]]), shape)[0]
            F_rc[p] -= mom
            T_rc[p] -= np.cross(d, mom)
        for z, y, x, fr in fills:
            # Same extraction as at any node: u = (sum c f - F/2) / rho.
            ft_new[:, z, y, x] = fr
            rho[z, y, x] = fr.sum()
            u[:, z, y, x] = (CF.T @ fr - 0.5 * self.F_body[:, z, y, x]) / fr.sum()
        ft_new[:, owner1 != -1] = np.nan
        st.ft, st.rho, st.u = ft_new, rho, u
        st.P = P1
        st.F_h, st.T_h, st.F_c = F_h, T_h, F_c
        st.F_rc, st.T_rc = F_rc, T_rc
        st.owner = owner1
        pipe = (cfg.pipe_radius, cfg.pipe_cx, cfg.pipe_cy) if self.wall_solid is not None else None
        st.links = geo.build_links(owner1, P1.X, P1.r, shape, cfg.ibb_max_order, pipe)
        st.extra["uncovered"] = len(zz)
        st.step += 1

    def markers(self):
        """Marker positions, particle (-1 for the wall), lever arms, volumes."""
        cfg, P = self.cfg, self.state.P
        xl, own, arm, dV = ibm.sphere_markers(P.X, P.r, cfg.ibm_retraction, cfg.shape)
        if cfg.wall == "pipe_z":
            xp, dVp = ibm.pipe_markers(cfg.pipe_radius, cfg.ibm_retraction, cfg.pipe_cx, cfg.pipe_cy, cfg.shape[2])
            xl = np.concatenate([xl, xp])
            own = np.concatenate([own, np.full(len(xp), -1)])
            arm = np.concatenate([arm, np.zeros((len(xp), 3))])
            dV = np.concatenate([dV, dVp])
        return xl, own, arm, dV

    def _step_ibm(self):
        cfg, st = self.cfg, self.state
        shape = cfg.shape
        P = st.P
        f = col.stream_pull(st.ft)
        rho = col.density(f)
        u_star = (col.momentum(f) + 0.5 * self.F_body) / rho
        xl, own, arm, dV = self.markers()
        U_d = np.zeros((len(xl), 3))
        sph = own >= 0
        U_d[sph] = P.U[own[sph]] + np.cross(P.Om[own[sph]], arm[sph])
        f_ib, u_corr, F_l = ibm.multi_direct_forcing(u_star, rho, xl, U_d, dV, 1 + cfg.ibm_iters, shape)
        st.ft, st.rho, st.u = col.collide(f, self.F_body + f_ib, self.s)
        st.extra["f_ib"] = f_ib
        Iu, IL = ibm.inner_integrals(st.u, P.X, P.r, shape)
        F_h = np.zeros((P.n, 3))
        T_h = np.zeros((P.n, 3))
        np.add.at(F_h, own[sph], -F_l[sph] * dV[sph, None])
        np.add.at(T_h, own[sph], -np.cross(arm[sph], F_l[sph]) * dV[sph, None])
        F_h += Iu - st.Iu
        T_h += IL - st.IL
        F_c = self._contact()
        st.P = advance(P, F_h + F_c, T_h, shape)
        st.Iu, st.IL = Iu, IL
        st.F_h, st.T_h, st.F_c = F_h, T_h, F_c
        st.F_l = F_l
        st.step += 1
