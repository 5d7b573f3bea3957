"""ctypes binding of liblbm.so (declared in include/lbm.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels. PyTorch supplies the device workspace and the stream. The
binding refuses to work without the compiled library; there is no other
execution path.
"""
import ctypes
import dataclasses
from pathlib import Path

import numpy as np

_LIB_PATH = Path(__file__).resolve().parent / "liblbm.so"
_lib = None

BC_NONE, BC_IBB, BC_IBM = 0, 1, 2
STORE_F32, STORE_F16S = 0, 1
WALL_NONE, WALL_PIPE_Z = 0, 1
SET_STATE, RELEASE, SET_RIGID = 0, 1, 2
MOTION_FREE, MOTION_FIXED, MOTION_PRESCRIBED = 0, 1, 2
LATTICE_D3Q19, LATTICE_D3Q27 = 0, 1
PIPE_BUDGET_MOMENTS, PIPE_BUDGET_TERMS = 38, 13
KERNEL_CLASSES = ("stream_collide", "geometry", "ibb_links", "refill", "ibm_prepass", "ibm_forcing",
                  "particle", "stats", "corrector")
NPROF = len(KERNEL_CLASSES)


class LbmError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.lbm_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


class _CConfig(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double), ("s_q", ctypes.c_double),
        ("s_pi", ctypes.c_double), ("s_m", ctypes.c_double),
        ("body_force", ctypes.c_double * 3),
        ("bc", ctypes.c_int32), ("ibb_max_order", ctypes.c_int32),
        ("ibm_retraction", ctypes.c_double), ("ibm_iters", ctypes.c_int32),
        ("store", ctypes.c_int32), ("wall", ctypes.c_int32),
        ("pipe_radius", ctypes.c_double), ("pipe_cx", ctypes.c_double), ("pipe_cy", ctypes.c_double),
        ("max_particles", ctypes.c_int32), ("max_radius", ctypes.c_double),
        ("coll_restitution", ctypes.c_double), ("coll_tc_steps", ctypes.c_double),
        ("lattice", ctypes.c_int32), ("tau_bulk", ctypes.c_double),
    ]


class _CStats(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("n_nodes", ctypes.c_int64), ("n_fluid", ctypes.c_int64),
        ("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3),
        ("ke_raw", ctypes.c_double), ("ke_masked", ctypes.c_double), ("ke_fluid", ctypes.c_double),
        ("eps_raw", ctypes.c_double), ("eps_masked", ctypes.c_double), ("eps_fluid", ctypes.c_double),
        ("umax", ctypes.c_double), ("bulk_u", ctypes.c_double),
        ("particle_ke", ctypes.c_double), ("particle_ke_rot", ctypes.c_double),
        ("eps_fluid_corrected", ctypes.c_double), ("n_corrected", ctypes.c_int64),
    ]


STATS_MAX_BINS = 256


def lib() -> ctypes.CDLL:
    """Load liblbm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB_PATH.exists():
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with paper_1906_05448_amd/_build.py "
                           "(or __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(str(_LIB_PATH))
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    cfgp = ctypes.POINTER(_CConfig)
    sig = {
        "lbm_config_default": (None, [cfgp]),
        "lbm_workspace_size": (ctypes.c_int, [cfgp, ctypes.POINTER(SZ)]),
        "lbm_init": (ctypes.c_int, [cfgp, P, SZ, P, ctypes.POINTER(P)]),
        "lbm_set_fields": (ctypes.c_int, [P, P, P]),
        "lbm_set_fields_device": (ctypes.c_int, [P, P, P]),
        "lbm_step": (ctypes.c_int, [P, I32]),
        "lbm_get_fields": (ctypes.c_int, [P, P, P]),
        "lbm_get_fields_device": (ctypes.c_int, [P, P, P]),
        "lbm_sync": (ctypes.c_int, [P]),
        "lbm_step_count": (ctypes.c_int, [P, ctypes.POINTER(I64)]),
        "lbm_set_particles": (ctypes.c_int, [P, I32, P, P, P, P, P, I32, I32]),
        "lbm_get_particles": (ctypes.c_int, [P, P, P, P]),
        "lbm_particle_count": (ctypes.c_int, [P, ctypes.POINTER(I32)]),
        "lbm_state_size": (ctypes.c_int, [P, ctypes.POINTER(SZ)]),
        "lbm_get_state": (ctypes.c_int, [P, P, SZ]),
        "lbm_set_state": (ctypes.c_int, [P, P, SZ]),
        "lbm_forces": (ctypes.c_int, [P, P, P, P]),
        "lbm_link_count": (ctypes.c_int, [P, ctypes.POINTER(I64)]),
        "lbm_get_links": (ctypes.c_int, [P, I64, P, P, P, P, P, ctypes.POINTER(I64)]),
        "lbm_geometry_counts": (ctypes.c_int, [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]),
        "lbm_ibm_support": (ctypes.c_int, [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]),
        "lbm_stats": (ctypes.c_int, [P, I32, ctypes.c_double, ctypes.POINTER(_CStats), P]),
        "lbm_spectrum": (ctypes.c_int, [P, I32, I32, P, P]),
        "lbm_pipe_budget_reset": (ctypes.c_int, [P, ctypes.c_double]),
        "lbm_pipe_budget_add": (ctypes.c_int, [P]),
        "lbm_pipe_budget_read": (ctypes.c_int, [P, ctypes.POINTER(I32), ctypes.POINTER(I64), P, P]),
        "lbm_corrector_cells": (ctypes.c_int, [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, I64, P, P, P,
                                                ctypes.POINTER(I64)]),
        "lbm_corrector_labels": (ctypes.c_int, [P, P, I64, ctypes.c_double, I32, P]),
        "lbm_corrector_set": (ctypes.c_int, [P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
        "lbm_mlp_workspace_size": (SZ, []),
        "lbm_mlp_init": (ctypes.c_int, [P, SZ, P, P, ctypes.POINTER(P)]),
        "lbm_mlp_set_params": (ctypes.c_int, [P, P]),
        "lbm_mlp_get_params": (ctypes.c_int, [P, P]),
        "lbm_mlp_device_params": (P, [P]),
        "lbm_mlp_forward": (ctypes.c_int, [P, P, I64, P]),
        "lbm_mlp_gradient": (ctypes.c_int, [P, P, P, I64, ctypes.POINTER(ctypes.c_double), P]),
        "lbm_mlp_adam_step": (ctypes.c_int, [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
        "lbm_mlp_gradient_noalloc": (ctypes.c_int, [P, P, P, I64, P, P, P]),
        "lbm_mlp_sync": (ctypes.c_int, [P]),
        "lbm_mlp_destroy": (None, [P]),
        "lbm_set_overlap": (ctypes.c_int, [P, I32]),
        "lbm_profile_enable": (ctypes.c_int, [P, I32]),
        "lbm_profile_read": (ctypes.c_int, [P, P, P]),
        "lbm_destroy": (None, [P]),
        "lbm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


@dataclasses.dataclass
class Config:
    """Mirror of lbm_config; field meanings are documented in include/lbm.h."""
    nx: int = 32
    ny: int = 32
    nz: int = 32
    tau: float = 0.6
    s_e: float = 1.19
    s_eps: float = 1.4
    s_q: float = 1.2
    s_pi: float = 1.4
    s_m: float = 1.98
    body_force: tuple = (0.0, 0.0, 0.0)
    bc: int = BC_NONE
    ibb_max_order: int = 2
    ibm_retraction: float = 0.0
    ibm_iters: int = 2
    store: int = STORE_F32
    wall: int = WALL_NONE
    pipe_radius: float = 0.0
    pipe_cx: float = 0.0
    pipe_cy: float = 0.0
    max_particles: int = 0
    max_radius: float = 0.0
    coll_restitution: float = 0.97
    coll_tc_steps: float = 8.0
    lattice: int = LATTICE_D3Q19
    tau_bulk: float = 0.0

    def to_c(self) -> _CConfig:
        c = _CConfig()
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            if f.name == "body_force":
                c.body_force = (ctypes.c_double * 3)(*map(float, v))
            else:
                setattr(c, f.name, v)
        return c

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz


def _check(status: int, where: str) -> None:
    if status != 0:
        raise LbmError(status, where)


def _host_ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def workspace_size(cfg: Config) -> int:
    L = lib()
    n = ctypes.c_size_t()
    _check(L.lbm_workspace_size(ctypes.byref(cfg.to_c()), ctypes.byref(n)), "lbm_workspace_size")
    return n.value


class Lattice:
    """One simulation context on the current GPU.

    The workspace is a torch uint8 tensor owned by this object; all work runs
    on ``stream`` (default: torch's current stream)."""

    def __init__(self, cfg: Config, device=None, stream=None):
        import torch
        self._torch = torch
        self.cfg = cfg
        L = lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = workspace_size(cfg)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.lbm_init(ctypes.byref(cfg.to_c()), ctypes.c_void_p(self.workspace.data_ptr()),
                              ctypes.c_size_t(nbytes), ctypes.c_void_p(self.stream.cuda_stream),
                              ctypes.byref(h)), "lbm_init")
        self._h = h

    # -- fields ---------------------------------------------------------
    def set_fields(self, u, rho=None) -> None:
        """u: [3, nz, ny, nx] array-like (converted to FP32); rho optional."""
        N = self.cfg.n_nodes
        u32 = np.ascontiguousarray(np.asarray(u, dtype=np.float32).reshape(3, N))
        r32 = None if rho is None else np.ascontiguousarray(np.asarray(rho, np.float32).reshape(N))
        _check(lib().lbm_set_fields(self._h, _host_ptr(u32), None if r32 is None else _host_ptr(r32)),
               "lbm_set_fields")

    def set_fields_device(self, u, rho=None) -> None:
        """u: torch float32 CUDA tensor [3, nz, ny, nx], rho optional."""
        assert u.is_cuda and u.dtype == self._torch.float32 and u.is_contiguous()
        _check(lib().lbm_set_fields_device(self._h, ctypes.c_void_p(u.data_ptr()),
                                           None if rho is None else ctypes.c_void_p(rho.data_ptr())),
               "lbm_set_fields_device")

    def get_fields(self):
        """Returns (u [3, nz, ny, nx], rho [nz, ny, nx]) as float32 numpy."""
        nx, ny, nz = self.cfg.shape
        u = np.empty((3, nz, ny, nx), np.float32)
        rho = np.empty((nz, ny, nx), np.float32)
        _check(lib().lbm_get_fields(self._h, _host_ptr(u), _host_ptr(rho)), "lbm_get_fields")
        return u, rho

    def get_fields_device(self, u, rho=None) -> None:
        _check(lib().lbm_get_fields_device(self._h, ctypes.c_void_p(u.data_ptr()) if u is not None else None,
                                           None if rho is None else ctypes.c_void_p(rho.data_ptr())),
               "lbm_get_fields_device")

    # -- particles --------------------------------------------------------
    def set_particles(self, x, radius, u=None, omega=None, rho_p=None, mode=SET_STATE,
                      motion=MOTION_FREE) -> None:
        x = np.ascontiguousarray(np.atleast_2d(np.asarray(x, np.float64)))
        n = x.shape[0]
        rad = np.ascontiguousarray(np.broadcast_to(np.asarray(radius, np.float64), (n,)))

        def opt(a, shape):
            return None if a is None else np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), shape))

        uu, ww, rr = opt(u, (n, 3)), opt(omega, (n, 3)), opt(rho_p, (n,))
        self._particles_keep = (x, rad, uu, ww, rr)
        _check(lib().lbm_set_particles(self._h, n, _host_ptr(x), None if uu is None else _host_ptr(uu),
                                       None if ww is None else _host_ptr(ww), _host_ptr(rad),
                                       None if rr is None else _host_ptr(rr), int(mode), int(motion)),
               "lbm_set_particles")
        self.n_particles = n

    def particle_count(self) -> int:
        n = ctypes.c_int32()
        _check(lib().lbm_particle_count(self._h, ctypes.byref(n)), "lbm_particle_count")
        return n.value

    # -- checkpoint -----------------------------------------------------
    def get_state(self) -> np.ndarray:
        """The context's state blob (lbm_get_state) as a uint8 array."""
        n = ctypes.c_size_t()
        _check(lib().lbm_state_size(self._h, ctypes.byref(n)), "lbm_state_size")
        blob = np.empty(n.value, np.uint8)
        _check(lib().lbm_get_state(self._h, _host_ptr(blob), n.value), "lbm_get_state")
        return blob

    def set_state(self, blob) -> None:
        """Restores a blob of get_state() (lbm_set_state)."""
        b = np.ascontiguousarray(np.asarray(blob, np.uint8))
        _check(lib().lbm_set_state(self._h, _host_ptr(b), b.size), "lbm_set_state")
        self.n_particles = self.particle_count()

    def get_particles(self):
        n = getattr(self, "n_particles", 0)
        X, U, W = (np.zeros((n, 3)) for _ in range(3))
        _check(lib().lbm_get_particles(self._h, _host_ptr(X), _host_ptr(U), _host_ptr(W)), "lbm_get_particles")
        return X, U, W

    def forces(self):
        """(hydrodynamic force, torque, contact force), each (np, 3)."""
        n = getattr(self, "n_particles", 0)
        F, T, Fc = (np.zeros((n, 3)) for _ in range(3))
        _check(lib().lbm_forces(self._h, _host_ptr(F), _host_ptr(T), _host_ptr(Fc)), "lbm_forces")
        return F, T, Fc

    def links(self):
        """Boundary links: dict of node (L, 3) xyz, dir (L, 3), particle (L,),
        q (L,) float32, scheme (L,)."""
        n = ctypes.c_int64()
        _check(lib().lbm_link_count(self._h, ctypes.byref(n)), "lbm_link_count")
        cap = n.value
        node = np.zeros((cap, 3), np.int32)
        d = np.zeros((cap, 3), np.int32)
        p = np.zeros(cap, np.int32)
        q = np.zeros(cap, np.float32)
        s = np.zeros(cap, np.int32)
        got = ctypes.c_int64()
        _check(lib().lbm_get_links(self._h, cap, _host_ptr(node), _host_ptr(d), _host_ptr(p), _host_ptr(q),
                                   _host_ptr(s), ctypes.byref(got)), "lbm_get_links")
        k = got.value
        return {"node": node[:k], "dir": d[:k], "particle": p[:k], "q": q[:k], "scheme": s[:k]}

    def geometry_counts(self):
        """(solid nodes, boundary links) of the current geometry."""
        s, l = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().lbm_geometry_counts(self._h, ctypes.byref(s), ctypes.byref(l)), "lbm_geometry_counts")
        return s.value, l.value

    def ibm_support(self):
        """(support nodes, shared nodes) of the immersed boundary."""
        s, h = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().lbm_ibm_support(self._h, ctypes.byref(s), ctypes.byref(h)), "lbm_ibm_support")
        return s.value, h.value

    def stats(self, nbins: int = 32, bin_width: float = 0.25) -> dict:
        """Statistics of the current snapshot (lbm_stats): a dict with the
        lbm_stats_t fields (momentum as an array) and "hist" [6][nbins]
        (count, sum 1/2|u|^2, sum eps, sum u_z, sum u_z^2, sum corrected eps
        per distance bin)."""
        out = _CStats()
        hist = np.zeros((6, max(int(nbins), 0)), np.float64)
        _check(lib().lbm_stats(self._h, int(nbins), float(bin_width), ctypes.byref(out),
                               hist.ctypes.data_as(ctypes.c_void_p) if nbins > 0 else None), "lbm_stats")
        d = {name: getattr(out, name) for name, _ in _CStats._fields_}
        d["momentum"] = np.array(list(out.momentum))
        d["hist"] = hist
        return d

    def spectrum(self, kmax: int, masked: bool = True):
        """(k, E, D) for shells k = 0 .. kmax of the current field
        (lbm_spectrum): energy spectrum and dissipation spectrum 2 nu k^2 E."""
        E = np.zeros(int(kmax) + 1, np.float64)
        D = np.zeros(int(kmax) + 1, np.float64)
        _check(lib().lbm_spectrum(self._h, 1 if masked else 0, int(kmax), _host_ptr(E), _host_ptr(D)),
               "lbm_spectrum")
        return np.arange(int(kmax) + 1, dtype=np.float64), E, D

    def pipe_budget_reset(self, bin_width: float) -> None:
        _check(lib().lbm_pipe_budget_reset(self._h, float(bin_width)), "lbm_pipe_budget_reset")

    def pipe_budget_add(self) -> None:
        _check(lib().lbm_pipe_budget_add(self._h), "lbm_pipe_budget_add")

    def pipe_budget_read(self):
        """(snapshots, moments [38, nbins], terms [13, nbins]) of the pipe's
        TKE budget accumulator (lbm_pipe_budget_read)."""
        nb, ns = ctypes.c_int32(), ctypes.c_int64()
        _check(lib().lbm_pipe_budget_read(self._h, ctypes.byref(nb), ctypes.byref(ns), None, None),
               "lbm_pipe_budget_read")
        M = np.zeros((PIPE_BUDGET_MOMENTS, nb.value), np.float64)
        T = np.zeros((PIPE_BUDGET_TERMS, nb.value), np.float64)
        _check(lib().lbm_pipe_budget_read(self._h, ctypes.byref(nb), ctypes.byref(ns), _host_ptr(M), _host_ptr(T)),
               "lbm_pipe_budget_read")
        return ns.value, M, T

    # -- gradient corrector ---------------------------------------------
    def corrector_cells(self, u_rms, d_min=0.0, d_max=10.0, cap=None, features=True):
        """(nodes int32, spheres int32, features bf16 [n, 96] or None) of the
        interface cells, as torch CUDA tensors."""
        t = self._torch
        if cap is None:
            n = ctypes.c_int64()
            st = lib().lbm_corrector_cells(self._h, d_min, d_max, u_rms, 0, None, None, None, ctypes.byref(n))
            if st not in (0, -3):
                _check(st, "lbm_corrector_cells")
            cap = n.value
        node = t.empty(max(cap, 1), dtype=t.int32, device=self.device)
        part = t.empty(max(cap, 1), dtype=t.int32, device=self.device)
        x = t.empty((max(cap, 1), MLP_IN_STRIDE), dtype=t.bfloat16, device=self.device) if features else None
        n = ctypes.c_int64()
        _check(lib().lbm_corrector_cells(self._h, d_min, d_max, u_rms, cap, _dev(node), _dev(part),
                                         _dev(x) if features else None, ctypes.byref(n)), "lbm_corrector_cells")
        k = n.value
        return node[:k], part[:k], (x[:k] if features else None)

    def corrector_labels(self, nodes, u_rms, subtract_from=None):
        """[n, 16] float32 CUDA labels at the given nodes (int32 CUDA tensor);
        with subtract_from (a label tensor, updated in place) its entries
        minus this lattice's labels."""
        t = self._torch
        n = int(nodes.shape[0])
        if subtract_from is None:
            out = t.empty((max(n, 1), MLP_OUT_STRIDE), dtype=t.float32, device=self.device)
        else:
            out = subtract_from
            assert out.is_contiguous() and out.dtype == t.float32 and out.shape == (n, MLP_OUT_STRIDE)
        _check(lib().lbm_corrector_labels(self._h, _dev(nodes) if n else None, n, u_rms,
                                          0 if subtract_from is None else 1, _dev(out) if n else None),
               "lbm_corrector_labels")
        return out[:n]

    def corrector_set(self, mlp=None, d_min=0.0, d_max=10.0, u_rms=0.03) -> None:
        """Attach an Mlp for stats() (None detaches); keeps a reference."""
        self._corrector = mlp
        ptr = lib().lbm_mlp_device_params(mlp._h) if mlp is not None else None
        _check(lib().lbm_corrector_set(self._h, ptr, d_min, d_max, u_rms), "lbm_corrector_set")

    # -- time stepping -------------------------------------------------
    def step(self, n: int = 1) -> None:
        _check(lib().lbm_step(self._h, int(n)), "lbm_step")

    def sync(self) -> None:
        _check(lib().lbm_sync(self._h), "lbm_sync")

    @property
    def step_count(self) -> int:
        s = ctypes.c_int64()
        _check(lib().lbm_step_count(self._h, ctypes.byref(s)), "lbm_step_count")
        return s.value

    # -- kernel timing ----------------------------------------------------
    def set_overlap(self, on: bool = True) -> None:
        """Particle stage and next geometry beside the stream-collide kernel
        on a second stream (lbm_set_overlap)."""
        _check(lib().lbm_set_overlap(self._h, 1 if on else 0), "lbm_set_overlap")

    def profile_enable(self, on: bool = True) -> None:
        _check(lib().lbm_profile_enable(self._h, 1 if on else 0), "lbm_profile_enable")

    def profile_read(self):
        """Returns {class name: (total ms, launches)} since the last read."""
        ms = np.zeros(NPROF, np.float64)
        n = np.zeros(NPROF, np.int64)
        _check(lib().lbm_profile_read(self._h, _host_ptr(ms), _host_ptr(n)), "lbm_profile_read")
        return {name: (float(ms[k]), int(n[k])) for k, name in enumerate(KERNEL_CLASSES)}

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MLP_IN, MLP_IN_STRIDE, MLP_OUT, MLP_OUT_STRIDE, MLP_PARAMS = 85, 96, 9, 16, 10249


def _dev(t):
    return ctypes.c_void_p(t.data_ptr())


class Mlp:
    """The gradient-corrector network on the current GPU (lbm_mlp_*).

    Features are torch bfloat16 CUDA tensors [n, 96]; targets and outputs
    float32 [n, 16]. Parameters are a float vector of 10,249 entries."""

    def __init__(self, params, device=None, stream=None):
        import torch
        self._torch = torch
        L = lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = L.lbm_mlp_workspace_size()
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        p = np.ascontiguousarray(np.asarray(params, np.float32).reshape(MLP_PARAMS))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.lbm_mlp_init(_dev(self.workspace), ctypes.c_size_t(nbytes), _host_ptr(p),
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "lbm_mlp_init")
        self._h = h

    def set_params(self, params) -> None:
        p = np.ascontiguousarray(np.asarray(params, np.float32).reshape(MLP_PARAMS))
        _check(lib().lbm_mlp_set_params(self._h, _host_ptr(p)), "lbm_mlp_set_params")

    def params(self) -> np.ndarray:
        p = np.empty(MLP_PARAMS, np.float32)
        _check(lib().lbm_mlp_get_params(self._h, _host_ptr(p)), "lbm_mlp_get_params")
        return p

    def _rows(self, x):
        t = self._torch
        assert x.is_cuda and x.dtype == t.bfloat16 and x.is_contiguous() and x.shape[-1] == MLP_IN_STRIDE
        return x.shape[0]

    def forward(self, x):
        n = self._rows(x)
        y = self._torch.empty((n, MLP_OUT_STRIDE), dtype=self._torch.float32, device=self.device)
        _check(lib().lbm_mlp_forward(self._h, _dev(x) if n else None, n, _dev(y) if n else None), "lbm_mlp_forward")
        return y

    def gradient(self, x, t, want_grad=False):
        """(loss, gradient or None) at the current parameters."""
        n = self._rows(x)
        assert t.is_cuda and t.dtype == self._torch.float32 and t.is_contiguous() and t.shape == (n, MLP_OUT_STRIDE)
        loss = ctypes.c_double()
        g = np.empty(MLP_PARAMS, np.float32) if want_grad else None
        _check(lib().lbm_mlp_gradient(self._h, _dev(x), _dev(t), n, ctypes.byref(loss),
                                      _host_ptr(g) if want_grad else None), "lbm_mlp_gradient")
        return loss.value, g

    def gradient_noalloc(self, x, t, grad, loss_sum, stream=None) -> None:
        """lbm_mlp_gradient_noalloc at this network's parameters: the gradient
        into grad (float32 CUDA [10249]) and the summed squared error into
        loss_sum (float64 CUDA [1]), with no allocation by the library."""
        n = self._rows(x)
        st = stream if stream is not None else self.stream
        _check(lib().lbm_mlp_gradient_noalloc(lib().lbm_mlp_device_params(self._h), _dev(x), _dev(t), n, _dev(grad),
                                              _dev(loss_sum), ctypes.c_void_p(st.cuda_stream)),
               "lbm_mlp_gradient_noalloc")

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
        _check(lib().lbm_mlp_adam_step(self._h, lr, beta1, beta2, eps), "lbm_mlp_adam_step")

    def sync(self) -> None:
        _check(lib().lbm_mlp_sync(self._h), "lbm_mlp_sync")

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().lbm_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
