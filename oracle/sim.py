"""Time-stepping driver of the FP64 oracle.

State at integer step n: post-collision populations f~(x, n) on every node
(fluid nodes only for interpolated bounce-back; solid nodes hold NaN so that
any read of them shows up), plus the particle state.

Periodic box, one step n -> n+1 without particles:
  1. pull streaming f_i(x) = f~_i(x - c_i)                       (collide.stream_pull)
  2. MRT + Guo collision under the body force rho*g (Sec. 2.1)    (collide.collide)
The macroscopic fields of step n+1 are the density and the half-force
velocity used in that collision.
"""
from dataclasses import dataclass, field

import numpy as np

from . import collide as col
from .lattice import DEFAULT_RATES, relaxation_vector


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
    extra: dict = field(default_factory=dict)


class Sim:
    """Plain FP64 reference run of the method."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        self.s = cfg.rates()
        zyx = cfg.zyx
        self.F_body = np.broadcast_to(np.asarray(cfg.body_force, np.float64).reshape(3, 1, 1, 1),
                                      (3,) + zyx).copy()
        rho = np.ones(zyx)
        u = np.zeros((3,) + zyx)
        self.state = State(ft=col.equilibrium(rho, u), rho=rho, u=u)

    # -- fields -----------------------------------------------------------
    def set_fields(self, u, rho=None):
        zyx = self.cfg.zyx
        u = np.asarray(u, np.float64).reshape((3,) + zyx)
        rho = np.ones(zyx) if rho is None else np.asarray(rho, np.float64).reshape(zyx)
        self.state = State(ft=col.equilibrium(rho, u), rho=rho.copy(), u=u.copy())

    def fields(self):
        return self.state.u, self.state.rho

    # -- stepping ---------------------------------------------------------
    def step(self, n: int = 1):
        for _ in range(n):
            self._step_plain()

    def _step_plain(self):
        st = self.state
        f = col.stream_pull(st.ft)
        st.ft, st.rho, st.u = col.collide(f, self.F_body, self.s)
        st.step += 1
