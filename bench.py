#!/usr/bin/env python3
"""Throughput of the lattice Boltzmann particle-resolved hot path on one MI355X.

Workload (production case): 512^3 periodic decaying isotropic turbulence,
D3Q19 MRT, tau 0.52, seeded random-phase field with E(k) ~ k^4 exp(-2 (k/4)^2)
and u_rms 0.03, 6250 freely moving spheres of radius 8 (volume fraction
~10%, density ratio 4 as in the paper's case) released into the field
(velocity = fluid average over the particle, zero spin), soft-sphere
contacts. A step is one full lbm_step: boundary treatment, fused stream +
collide, particle forces and motion, geometry rebuild and refilling; every
--stats-every steps the FP64 statistics (lbm_stats) run inside the timed
region too, with the learned corrector in the ibmc variant (trained at
start on paired 64^3 runs through the same library).

Prints ONE JSON line on stdout (progress goes to stderr):
  value        million lattice-node updates per second (MLUPS) over all N
               nodes for the headline variant, inputs resident in HBM
  roofline     the dominant kernel (fused stream + collide): algorithmic
               bytes per launch / its average duration, timed with HIP events
               on the launch stream, against the 8 TB/s HBM peak
  cpu_baseline the FP64 oracle, single-threaded, on a bounded sample of the
               same recipe on this host
  variants     every variant measured (boundary treatment x storage, and
               the bounce-back and immersed-boundary FP16 steps with the
               particle stage and the next geometry overlapped with the
               stream-collide kernel on a second stream: "-ov")
  corrector    training throughput of the corrector network, MFMA
               utilisation of its kernels, and its held-out gain
  cpu_baseline also carries error_vs_fp64: relative L2 of the FP32 and FP16
               velocity fields against the oracle on the same sample
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS at 512^3 particle-laden D3Q19 (%HBM roofline), FP32/FP16 vs FP64 error"
HBM_PEAK_GBS = 8000.0
U_RMS = 0.03
TAU = 0.52
RADIUS = 8.0
RHO_P = 4.0            # particle/fluid density ratio of the paper's case (Sec. 3.1, Table 2)
IBM_RD = 0.4           # Breugem retraction, the variant the paper recommends
MIN_GAP = 2.0          # centre distance >= 2r + 2 at placement


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stream_collide_traffic_512cubed.md")
# the kernels and the population layout (array stride and pad) they run on
TRAFFIC_SOURCES = ("paper_1906_05448_amd/csrc/dense.hip", "paper_1906_05448_amd/csrc/d3q19.hpp",
                   "paper_1906_05448_amd/csrc/internal.hpp")
PIPE27_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pipe27_traffic_160x160x480.md")
PIPE27_SOURCES = ("paper_1906_05448_amd/csrc/d3q27.hip", "paper_1906_05448_amd/csrc/d3q27.hpp",
                  "paper_1906_05448_amd/csrc/internal.hpp")


def kernel_source_hash(sources=None):
    import hashlib
    h = hashlib.sha256()
    for f in sources or TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _traffic_record(path, tag, sources, variant):
    """traffic_bytes_per_launch of `variant` from a committed counter summary
    whose source_sha256 `tag` line matches the current kernel sources."""
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    rec = {}
    for ln in lines:
        parts = ln.strip().strip("`").split()
        if len(parts) == 3 and parts[0] in ("traffic_bytes_per_launch", "source_sha256"):
            rec[(parts[0], parts[1])] = parts[2]
    if rec.get(("source_sha256", tag)) != kernel_source_hash(sources):
        return None
    v = rec.get(("traffic_bytes_per_launch", variant))
    return int(v) if v is not None else None


def recorded_traffic(variant, n, particles):
    """HBM bytes per launch of the fused kernel from the committed counter
    summary, if it was taken on the current kernel source and this workload
    (512^3, 6250 spheres), else None."""
    if n != 512 or particles != 6250:
        return None
    return _traffic_record(TRAFFIC_FILE, "dense", TRAFFIC_SOURCES, variant)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--n", type=int, default=512, help="lattice edge (production: 512)")
    p.add_argument("--particles", type=int, default=6250)
    p.add_argument("--variants",
                   default="ibb-f16s,ibb-f32,ibm-f16s,ibmc-f16s,ibm-f32,none-f16s,none-f32,ibb-f16s-ov,ibm-f16s-ov",
                   help="comma list of <bc>-<store>[-ov], bc in ibb|ibm|ibmc (immersed boundary with the learned "
                        "corrector in the statistics)|none, store in f16s|f32, -ov: the particle stage and the "
                        "next geometry on a second stream beside the stream-collide kernel (lbm_set_overlap); "
                        "the first is the headline")
    p.add_argument("--stats-every", type=int, default=100, help="steps between lbm_stats calls (0: none)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--pipe", action="store_true",
                   help="time the 160x160x480 pipe (R = 74.5, linear bounce-back wall, FP32) and one snapshot of "
                        "its component TKE budget instead of the headline workload")
    p.add_argument("--pipe-lattice", type=int, choices=(19, 27), default=27,
                   help="pipe solver lattice: 27 (the paper's pipe model, one relaxation parameter) or 19 (MRT)")
    return p.parse_args()


def advance(lat, steps, every):
    """steps time steps with lbm_stats after every `every` steps, and after the
    last step when fewer than `every` are timed, so the statistics (and the
    corrector) always run inside the timed region; returns (the last
    statistics or None, the number of statistics calls)."""
    s = None
    done = calls = 0
    while done < steps:
        k = steps - done if every <= 0 else min(every, steps - done)
        lat.step(k)
        done += k
        if every > 0 and (done % every == 0 or (done == steps and calls == 0)):
            s = lat.stats(nbins=32)
            calls += 1
    return s, calls


def step_bytes(bc, s, N, fluid, links, support, stats_per_step=0.0):
    """Algorithmic HBM bytes of one step (the method's traffic, not the
    implementation's): every fluid node's 19 populations read and written
    once; bounce-back adds the solid bitmask and 16 bytes of link data per
    link (written by the geometry, read by the link pass); the immersed
    boundary adds per support node the pre-pass (19 populations read, the
    density and velocity written: 12 bytes), three forcing passes (12 bytes
    read, 24 bytes of force read-modify-write) and the force read by the
    collision (12 bytes). Statistics calls inside the timed steps add, per
    call and node, the velocity extraction (19 populations read, velocity
    and density written: 16 bytes), the key written (4 bytes) and the sums'
    reads of velocity, density and key (20 bytes), spread over the steps."""
    stats = int(stats_per_step * (38 * s + 40) * N)
    if bc == "ibb":
        return 38 * s * fluid + N // 8 + 16 * links + stats
    if bc in ("ibm", "ibmc"):
        return 38 * s * N + support * (19 * s + 12 + 3 * 36 + 12) + stats
    return 38 * s * N + stats


def run_variant(torch, lbm, n, bc, store, u0_dev, X, steps, warmup, every, corr=None, overlap=False):
    cfg = lbm.Config(nx=n, ny=n, nz=n, tau=TAU, store=store, bc=bc, ibm_retraction=IBM_RD,
                     max_particles=len(X) if bc != lbm.BC_NONE else 0, max_radius=RADIUS)
    lat = lbm.Lattice(cfg)
    lat.set_overlap(overlap)
    lat.set_fields_device(u0_dev)
    if bc != lbm.BC_NONE and len(X):
        lat.set_particles(X, RADIUS, rho_p=RHO_P, mode=lbm.RELEASE, motion=lbm.MOTION_FREE)
    if corr is not None:
        lat.corrector_set(corr, 0.0, 10.0, U_RMS)
    solid, links = lat.geometry_counts() if bc == lbm.BC_IBB else (0, 0)
    support, shared = lat.ibm_support() if bc == lbm.BC_IBM else (0, 0)
    lat.step(warmup)
    lat.sync()
    stream = lat.stream
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    st, stats_calls = advance(lat, steps, every)
    t1.record(stream)
    torch.cuda.synchronize()
    lat.sync()
    ms = t0.elapsed_time(t1)
    # Second pass with per-kernel events for the roofline of the dominant kernel.
    lat.profile_enable(True)
    advance(lat, steps, every)
    prof = lat.profile_read()
    lat.profile_enable(False)
    lat.sync()
    # masked energy and dissipation spectra of the final field (every shell),
    # a statistics call outside the stepping loop
    spec_ms = None
    if n & (n - 1) == 0:
        kmax = int(np.floor(np.sqrt(3.0) * n / 2 + 0.5))
        lat.spectrum(kmax)
        t0.record(stream)
        for _ in range(3):
            lat.spectrum(kmax)
        t1.record(stream)
        torch.cuda.synchronize()
        spec_ms = t0.elapsed_time(t1) / 3
    lat.close()
    del lat
    torch.cuda.empty_cache()
    N = n ** 3
    s = 4 if store == lbm.STORE_F32 else 2
    k_ms, k_n = prof["stream_collide"]
    k_avg = k_ms / max(k_n, 1)
    # Algorithmic bytes of the fused kernel: 19 populations read and written
    # per node (every node is updated; a bounce-back sphere is narrower than
    # one 64-node wavefront row, so fluid-only updates would touch the same
    # cache lines), plus the support bitmask and rank words with the immersed
    # boundary (8 bytes per 32 nodes).
    alg_bytes = 38 * s * N + (N // 4 if bc == lbm.BC_IBM else 0)
    achieved = alg_bytes / (k_avg * 1e-3) / 1e9
    out = dict(ms_per_step=ms / steps, mlups=N * steps / (ms * 1e-3) / 1e6,
               kernel_avg_ms=k_avg, kernel_launches=k_n, alg_bytes=alg_bytes, achieved_gbs=achieved,
               solid_nodes=solid, links=links, support_nodes=support, shared_support_nodes=shared,
               stats_calls_timed=stats_calls,
               kernels_ms_per_step={k: v[0] / steps for k, v in prof.items() if v[1]},
               spectrum_ms=spec_ms)
    if st is not None:
        out["stats"] = {k: st[k] for k in ("ke_masked", "eps_fluid", "eps_fluid_corrected", "n_corrected",
                                            "particle_ke")}
    return out


def copy_calibration(torch):
    """A plain device-to-device copy of 2 GiB (the runtime's copy kernel):
    the achievable streaming bandwidth next to the 8 TB/s peak, and the
    known-size reference for scaling HBM byte counters."""
    n = 1 << 29
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record(stream)
    for _ in range(reps):
        b.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    moved = 2 * 4 * n
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_read_per_copy": 4 * n, "bytes_written_per_copy": 4 * n, "ms": round(ms, 4),
            "gbs": round(moved / (ms * 1e-3) / 1e9, 1)}


def train_corrector(torch, lbm):
    """Trains the gradient corrector on paired 64^3 runs (seeds 0-1) through
    the library and measures its held-out gain (seed 7) and the throughput
    and MFMA utilisation of the network kernels."""
    from paper_1906_05448_amd import corrector
    import synth
    cfg = corrector.PairConfig()
    parts = [corrector.paired_samples(cfg, s) for s in (0, 1)]
    x = torch.cat([p[0] for p in parts])
    t = torch.cat([p[1] for p in parts])
    net = lbm.Mlp(synth.mlp_initial_params(0))
    steps, batch = 1500, 4096
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    losses = corrector.train(net, x, t, steps=steps, batch=batch, lr=1e-3, seed=0)
    e1.record(stream)
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1)
    # network kernels alone: gradient (forward + backward) and forward of one
    # large batch, timed on the stream with no host work in between
    xb, tb = x[:batch].contiguous(), t[:batch].contiguous()
    xf = x.repeat(64, 1).contiguous()
    e0.record(stream)
    for _ in range(50):
        if lbm.lib().lbm_mlp_gradient(net._h, lbm._dev(xb), lbm._dev(tb), batch, None, None) != 0:
            raise RuntimeError("lbm_mlp_gradient failed")
    e1.record(stream)
    torch.cuda.synchronize()
    grad_ms = e0.elapsed_time(e1) / 50
    e0.record(stream)
    for _ in range(10):
        y = net.forward(xf)
    e1.record(stream)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 10
    # the gradient on a large batch (about 1 M samples): the kernels' own
    # throughput, which a 4 096-sample training batch does not fill
    big = min(1 << 20, xf.shape[0])
    xg = xf[:big].contiguous()
    tg = t.repeat((big + t.shape[0] - 1) // t.shape[0], 1)[:big].contiguous()
    e0.record(stream)
    for _ in range(10):
        if lbm.lib().lbm_mlp_gradient(net._h, lbm._dev(xg), lbm._dev(tg), big, None, None) != 0:
            raise RuntimeError("lbm_mlp_gradient failed")
    e1.record(stream)
    torch.cuda.synchronize()
    grad_big_ms = e0.elapsed_time(e1) / 10
    xe, te, tbe = corrector.paired_samples(cfg, 7)
    y = net.forward(xe)
    nu = (cfg.tau - 0.5) / 3

    def eps(G):  # 2 nu s_ij s_ij per row of u_rms-scaled gradients (evaluation only)
        G = G[:, :9].double().reshape(-1, 3, 3) * cfg.u_rms
        S = 0.5 * (G + G.transpose(1, 2))
        return 2 * nu * (S * S).sum((1, 2))

    e_ref, e_ibm, e_cor = eps(te + tbe), eps(tbe), eps(tbe + y)
    err_plain = float(torch.linalg.norm(e_ibm - e_ref) / torch.linalg.norm(e_ref))
    err_corr = float(torch.linalg.norm(e_cor - e_ref) / torch.linalg.norm(e_ref))
    # matrix-core work issued per sample (padded shapes 96-64-64-16): forward
    # 2 (96*64 + 64*64 + 64*16) flop; the gradient adds the weight gradients
    # (the same products) and the back-propagation through W3 (out padded to
    # 32) and W2: 2 (32*64 + 64*64) more (the MFMA op counters give both)
    fwd_flop = 2 * (96 * 64 + 64 * 64 + 64 * 16)
    grad_flop = 2 * fwd_flop + 2 * (32 * 64 + 64 * 64)
    peak = 2.5e15
    info = dict(train_samples=int(x.shape[0]), steps=steps, batch=batch,
                train_samples_per_s=round(steps * batch / (train_ms * 1e-3), 1),
                loss_first=round(float(losses[:10].mean()), 5), loss_last=round(float(losses[-100:].mean()), 5),
                heldout_eps_rel_l2_plain_ibm=round(err_plain, 4), heldout_eps_rel_l2_corrected=round(err_corr, 4),
                gradient_kernel_ms_batch4096=round(grad_ms, 4),
                gradient_mfma_util=round(grad_flop * batch / (grad_ms * 1e-3) / peak, 5),
                gradient_kernel_ms_large=round(grad_big_ms, 4), gradient_large_batch=int(big),
                gradient_large_mfma_util=round(grad_flop * big / (grad_big_ms * 1e-3) / peak, 5),
                forward_ms=round(fwd_ms, 4), forward_samples=int(xf.shape[0]),
                forward_mfma_util=round(fwd_flop * xf.shape[0] / (fwd_ms * 1e-3) / peak, 5))
    log(f"bench: corrector {info}")
    return net, info


def host_description():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def _oracle_sample(bc, threads, budget_s):
    """The FP64 oracle on a 64^3 box of the production recipe (12 released
    spheres of radius 8, ~10% volume fraction, density ratio 4) with the
    given no-slip treatment, timed over about budget_s seconds of stepping
    with the numerical libraries limited to `threads` threads (None: their
    default). Returns (sim, u0, X, steps timed, seconds, threads used)."""
    from threadpoolctl import threadpool_info, threadpool_limits

    import synth
    from oracle.sim import RELEASE, Config as OConfig, Sim as OSim
    n = 64
    spec = synth.hit_spectrum(seed=0, u_rms=U_RMS)
    u0 = synth.hit_field(spec, (n, n, n))
    X = synth.random_spheres(12, (n, n, n), 2 * RADIUS + MIN_GAP, seed=0)
    with threadpool_limits(limits=threads):
        used = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
        sim = OSim(OConfig(shape=(n, n, n), tau=TAU, bc=bc, ibm_retraction=IBM_RD))
        sim.set_fields(u0)
        sim.set_particles(X, r=np.full(len(X), RADIUS), rho_p=np.full(len(X), RHO_P), mode=RELEASE)
        sim.step(1)
        t = time.perf_counter()
        sim.step(1)
        one = time.perf_counter() - t
        steps = max(2, min(200, int(budget_s / max(one, 1e-3))))
        t = time.perf_counter()
        sim.step(steps)
        dt = time.perf_counter() - t
    return sim, u0, X, steps, dt, used


def cpu_baseline():
    """The FP64 oracle on a bounded sample of the same recipe (a 64^3 box,
    12 released spheres of radius 8, bounce-back), timed with the numerical
    libraries on all usable cores and on one core: about 10 s of CPU work
    each. The same sample with bounce-back and with the immersed boundary
    also gives the GPU's FP32 and FP16 error against FP64."""
    n = 64
    host = host_description()
    sim, u0, X, steps, dt, used = _oracle_sample("ibb", None, 10.0)
    _, _, _, steps1, dt1, _ = _oracle_sample("ibb", 1, 10.0)
    out = dict(value=n ** 3 * steps / dt / 1e6, unit="MLUPS", cores=used, kind="oracle",
               sample=f"{n}^3 box of the same recipe with 12 spheres r=8 (bounce-back, FP64 numpy oracle), "
                      f"{steps} steps in {dt:.1f} s with {used} threads",
               single_core={"value": n ** 3 * steps1 / dt1 / 1e6, "unit": "MLUPS", "cores": 1,
                            "sample": f"the same, {steps1} steps in {dt1:.1f} s"},
               host=host)
    err = {"ibb": gpu_error_vs_oracle(sim, u0, X, steps + 2, "ibb")}
    sim_m, u0m, Xm, steps_m, _, _ = _oracle_sample("ibm", None, 6.0)
    err["ibm"] = gpu_error_vs_oracle(sim_m, u0m, Xm, steps_m + 2, "ibm")
    out["error_vs_fp64"] = err
    return out


def gpu_error_vs_oracle(sim, u0, X, steps, bc):
    """The same sample on the GPU in FP32 and FP16 storage: relative L2 of the
    velocity over fluid nodes and relative error of the fluid dissipation
    against the FP64 oracle state (the metric's error column)."""
    from oracle import stats as ostats
    from paper_1906_05448_amd import lbm
    n = sim.cfg.shape[0]
    uo, ro = sim.fields()
    P = sim.state.P
    nu = (TAU - 0.5) / 3
    so = ostats.statistics(uo, ro, nu, sim.cfg.shape, P.X, P.U, P.Om, P.r, P.rho, nbins=0)
    fluid = sim.fluid_mask()
    res = {"steps": steps}
    for name, store in (("f32", lbm.STORE_F32), ("f16s", lbm.STORE_F16S)):
        lat = lbm.Lattice(lbm.Config(nx=n, ny=n, nz=n, tau=TAU, store=store,
                                     bc=lbm.BC_IBB if bc == "ibb" else lbm.BC_IBM, ibm_retraction=IBM_RD,
                                     max_particles=len(X), max_radius=RADIUS))
        lat.set_fields(u0)
        lat.set_particles(X, RADIUS, rho_p=RHO_P, mode=lbm.RELEASE, motion=lbm.MOTION_FREE)
        lat.step(steps)
        ug, _ = lat.get_fields()
        sg = lat.stats(nbins=0)
        Xg, Ug, _ = lat.get_particles()
        lat.close()
        du = (ug.astype(np.float64) - uo)[:, fluid]
        res[name] = {"u_rel_l2": float(np.linalg.norm(du) / np.linalg.norm(uo[:, fluid])),
                     "eps_fluid_rel": float(abs(sg["eps_fluid"] - so["eps_fluid"]) / so["eps_fluid"]),
                     "particle_U_rel_l2": float(np.linalg.norm(Ug - P.U) / np.linalg.norm(P.U))}
    return res


def run_pipe(torch, lbm, synth, steps, warmup, q=27):
    """The turbulent-pipe workload: steps per second, one TKE-budget snapshot
    (lbm_pipe_budget_add) and one statistics call, timed with HIP events on
    the library's stream; the fused stream-collide kernel's HBM roofline from
    the library's per-kernel events over a second pass."""
    shape, R, c = (160, 160, 480), 74.5, (79.5, 79.5)
    tau, F = 0.52, 7e-6
    cfg = lbm.Config(nx=shape[0], ny=shape[1], nz=shape[2], tau=tau, body_force=(0.0, 0.0, F), bc=lbm.BC_IBB,
                     ibb_max_order=1, wall=lbm.WALL_PIPE_Z, pipe_radius=R, pipe_cx=c[0], pipe_cy=c[1],
                     store=lbm.STORE_F32, lattice=lbm.LATTICE_D3Q27 if q == 27 else lbm.LATTICE_D3Q19)
    lat = lbm.Lattice(cfg)
    u0 = synth.pipe_initial_velocity(shape, R, c, 0.05, 0.05, seed=0)
    lat.set_fields(u0.astype(np.float32))
    lat.step(warmup)
    lat.sync()
    stream = lat.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / steps
    lat.profile_enable(True)
    lat.step(steps)
    prof = lat.profile_read()
    lat.profile_enable(False)
    lat.sync()
    sc_ms = prof["stream_collide"][0] / prof["stream_collide"][1]
    lat.pipe_budget_reset(0.5)
    lat.pipe_budget_add()  # warm
    t = []
    for what in ("budget", "stats"):
        e0.record(stream)
        for _ in range(3):
            lat.pipe_budget_add() if what == "budget" else lat.stats(nbins=32)
        e1.record(stream)
        torch.cuda.synchronize()
        t.append(e0.elapsed_time(e1) / 3)
    ns, M, T = lat.pipe_budget_read()
    lat.close()
    N = shape[0] * shape[1] * shape[2]
    gbs = 2 * q * 4 * N / (sc_ms * 1e-3) / 1e9   # every population read once and written once, FP32
    model = ("D3Q27, one relaxation parameter (BGK)" if q == 27 else "D3Q19 MRT")
    return {"metric": "pipe step time and TKE-budget snapshot time", "unit": "ms", "n_gpus": 1,
            "data": "synthetic", "dtype": "f32",
            "config": {"workload": f"160x160x480 pipe, R=74.5 along z, {model}, linear interpolated bounce-back "
                                   "wall, FP32 populations, tau 0.52, body force 7e-6, Poiseuille start + 5% noise",
                       "lattice": f"D3Q{q}", "budget_bin_width": 0.5, "budget_bins": int(M.shape[1])},
            "steps": steps, "warmup": warmup, "ms_per_step": round(step_ms, 4),
            "mlups": round(N / (step_ms * 1e-3) / 1e6, 1), "budget_add_ms": round(t[0], 4),
            "stats_ms": round(t[1], 4), "budget_snapshots": int(ns),
            "roofline": {"bound": "hbm", "kernel": f"stream_collide (D3Q{q})", "achieved": round(gbs, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "traffic": (_traffic_record(PIPE27_TRAFFIC_FILE, "d3q27", PIPE27_SOURCES, "pipe27")
                                     if q == 27 else None), "ms": round(sc_ms, 4)}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    from paper_1906_05448_amd import lbm

    torch.cuda.set_device(0)
    if args.pipe:
        print(json.dumps(run_pipe(torch, lbm, synth, args.steps, args.warmup, args.pipe_lattice)), flush=True)
        return
    n = args.n
    bcs = {"ibb": lbm.BC_IBB, "ibm": lbm.BC_IBM, "ibmc": lbm.BC_IBM, "none": lbm.BC_NONE}
    stores = {"f32": lbm.STORE_F32, "f16s": lbm.STORE_F16S}
    # name = boundary-storage[-ov]; "-ov": lbm_set_overlap on
    names = args.variants.split(",")
    variants = [v.split("-")[:2] for v in names]
    overlap = {v: v.endswith("-ov") for v in names}
    net, cinfo = None, None
    if any(bc == "ibmc" for bc, _ in variants):
        log("bench: training the gradient corrector on paired 64^3 runs")
        net, cinfo = train_corrector(torch, lbm)
    log(f"bench: {n}^3 seeded turbulence field and {args.particles} sphere centres")
    spec = synth.hit_spectrum(seed=0, u_rms=U_RMS)
    u0 = torch.from_numpy(synth.hit_field(spec, (n, n, n), dtype=np.float32)).cuda()
    X = synth.random_spheres(args.particles, (n, n, n), 2 * RADIUS + MIN_GAP, seed=0)
    copy = copy_calibration(torch)
    log(f"bench: device copy {copy}")
    results = {}
    for (bc, st), name in zip(variants, names):
        log(f"bench: variant {name}: warmup {args.warmup}, timed {args.steps} steps")
        results[name] = run_variant(torch, lbm, n, bcs[bc], stores[st], u0, X, args.steps, args.warmup,
                                    args.stats_every, net if bc == "ibmc" else None, overlap[name])
        r = results[name]
        log(f"bench: {name}: {r['mlups']:.0f} MLUPS, {r['ms_per_step']:.3f} ms/step, stream_collide "
            f"{r['kernel_avg_ms']:.3f} ms = {r['achieved_gbs']:.0f} GB/s; per step {r['kernels_ms_per_step']}")
    del u0
    head_name = names[0]
    head = results[head_name]
    hb, hs = variants[0]
    N = n ** 3
    for (bc, st), name in zip(variants, names):
        r = results[name]
        b = step_bytes(bc, 4 if st == "f32" else 2, N, N - r["solid_nodes"], r["links"], r["support_nodes"],
                       r["stats_calls_timed"] / args.steps)
        r["step_alg_bytes"] = b
        r["step_roofline_frac"] = b / (r["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS
    out = {
        "metric": METRIC,
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{n}^3 periodic decaying turbulence with {args.particles} released spheres "
                               f"r={RADIUS:g} (phi~10%), D3Q19 MRT tau {TAU}, u_rms {U_RMS}",
                   "lattice": [n, n, n], "particles": args.particles if hb != "none" else 0, "radius": RADIUS,
                   "density_ratio": RHO_P,
                   "boundary": {"ibb": "interpolated bounce-back (quadratic, fallback chain, refill)",
                                "ibm": f"immersed boundary, r_d={IBM_RD}, 1+2 forcing passes, Kempe inertia",
                                "ibmc": f"immersed boundary, r_d={IBM_RD}, with the learned gradient corrector",
                                "none": "no particles"}[hb],
                   "stats_every": args.stats_every,
                   "storage": {"f16s": "FP16 shifted populations, FP32 collision",
                               "f32": "FP32 shifted populations"}[hs]},
        "roofline": {"bound": "hbm", "achieved": round(head["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(head["achieved_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": recorded_traffic(head_name, n, args.particles),
                     "kernel": ("k_stream_collide_row" if n % 512 == 0 else "k_stream_collide_seg" if n % 2 == 0
                                else "k_stream_collide") if hs == "f16s"
                               else ("k_stream_collide_row32" if n % 512 == 0 else "k_stream_collide"),
                     "alg_bytes_per_launch": head["alg_bytes"],
                     "avg_launch_ms": round(head["kernel_avg_ms"], 4)},
        "step_roofline": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                          "alg_bytes_per_step": head["step_alg_bytes"],
                          "achieved": round(head["step_alg_bytes"] / (head["ms_per_step"] * 1e-3) / 1e9, 1),
                          "frac": round(head["step_roofline_frac"], 4),
                          "model": "whole step: fused stream-collide over the fluid nodes plus the boundary "
                                   "treatment's algorithmic bytes and the timed statistics calls' share "
                                   "(bench.step_bytes)"},
        "stream_copy": copy,
        "variants": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                     for k, v in results.items()},
    }
    if cinfo is not None:
        out["corrector"] = cinfo
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on a bounded CPU sample")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
