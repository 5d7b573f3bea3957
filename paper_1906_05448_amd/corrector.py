"""Training data and training loop of the near-surface gradient corrector.

Pairing (reading; the paper motivates a correction of the immersed-boundary
near-surface gradients, Sec. 3.2.1 and Sec. 4, without specifying one):
a bounce-back run (lattice A) carries the reference; from each of its
snapshots an immersed-boundary run (lattice B) starts with the same field
and the same particles, their interiors reset to the rigid-body motion;
both advance K steps with identical prescribed particle motion; the
features come from B at its interface cells and the labels from A at the
same cells. The network learns the correction of the plain immersed-
boundary gradient (B's own labels): the training target is A's labels minus
B's, and the corrected gradient is B's plain gradient plus u_rms times the
output. The plain gradient is the baseline the corrector has to beat.

Everything here drives the library through its C ABI (lattices, cells,
features, labels, network gradient and Adam); the host only picks seeds and
minibatch indices.
"""
from dataclasses import dataclass

import numpy as np

from . import lbm


@dataclass
class PairConfig:
    shape: tuple = (64, 64, 64)
    n_spheres: int = 6
    radius: float = 8.0
    r_d: float = 0.4            # immersed-boundary marker retraction
    tau: float = 0.52
    u_rms: float = 0.03
    snapshots: int = 3
    spinup: int = 60            # bounce-back steps before the first snapshot
    gap: int = 30               # bounce-back steps between snapshots
    K: int = 20                 # paired steps before sampling
    d_min: float = 0.0
    d_max: float = 10.0
    store: int = lbm.STORE_F32
    samples: int = 0            # > 0: that many cells per snapshot, drawn without replacement (seeded)


def _motion(n, radius, u_rms, rng):
    """Prescribed particle velocities and spins (seeded draws)."""
    U = rng.normal(0.0, 0.5 * u_rms, size=(n, 3))
    W = rng.normal(0.0, 0.5 * u_rms / radius, size=(n, 3))
    return U, W


def paired_samples(cfg: PairConfig, seed: int):
    """Features (bf16 [n, 96]), training targets (bounce-back minus plain
    immersed-boundary labels) and the plain labels (float32 [n, 16]) as torch
    CUDA tensors, from cfg.snapshots snapshots of one seeded run."""
    import torch

    import synth
    nx, ny, nz = cfg.shape
    spec = synth.hit_spectrum(seed=seed, u_rms=cfg.u_rms)
    u0 = synth.hit_field(spec, cfg.shape)
    X = synth.random_spheres(cfg.n_spheres, cfg.shape, 2 * cfg.radius + 2.0, seed=seed)
    U, W = _motion(cfg.n_spheres, cfg.radius, cfg.u_rms, np.random.default_rng(seed + 7919))
    common = dict(nx=nx, ny=ny, nz=nz, tau=cfg.tau, store=cfg.store, max_particles=cfg.n_spheres,
                  max_radius=cfg.radius)
    A = lbm.Lattice(lbm.Config(bc=lbm.BC_IBB, **common))
    B = lbm.Lattice(lbm.Config(bc=lbm.BC_IBM, ibm_retraction=cfg.r_d, **common))
    A.set_fields(u0)
    A.set_particles(X, cfg.radius, u=U, omega=W, mode=lbm.SET_RIGID, motion=lbm.MOTION_PRESCRIBED)
    A.step(cfg.spinup)
    xs, ts, tbs = [], [], []
    for s in range(cfg.snapshots):
        if s:
            A.step(cfg.gap)
        ua, ra = A.get_fields()
        Xa, _, _ = A.get_particles()
        B.set_fields(ua, ra)
        B.set_particles(Xa, cfg.radius, u=U, omega=W, mode=lbm.SET_RIGID, motion=lbm.MOTION_PRESCRIBED)
        A.step(cfg.K)
        B.step(cfg.K)
        nodes, _, x = B.corrector_cells(cfg.u_rms, cfg.d_min, cfg.d_max)
        if 0 < cfg.samples < nodes.shape[0]:
            gen = torch.Generator(device=nodes.device)
            gen.manual_seed(seed * 1000 + s)
            pick = torch.randperm(nodes.shape[0], device=nodes.device, generator=gen)[:cfg.samples]
            pick = pick.sort().values
            nodes = nodes.index_select(0, pick).contiguous()
            x = x.index_select(0, pick)
        xs.append(x.clone())
        target = A.corrector_labels(nodes, cfg.u_rms).clone()
        B.corrector_labels(nodes, cfg.u_rms, subtract_from=target)
        ts.append(target)
        tbs.append(B.corrector_labels(nodes, cfg.u_rms).clone())
    A.close()
    B.close()
    return torch.cat(xs), torch.cat(ts), torch.cat(tbs)


def train(net: "lbm.Mlp", x, t, steps: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0,
          beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """Adam on minibatches drawn uniformly with replacement (seeded); returns
    the loss of every step."""
    import torch
    gen = torch.Generator(device=x.device)
    gen.manual_seed(seed)
    n = x.shape[0]
    losses = []
    for _ in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), device=x.device, generator=gen)
        xb = x.index_select(0, idx).contiguous()
        tb = t.index_select(0, idx).contiguous()
        loss, _ = net.gradient(xb, tb)
        net.adam_step(lr, beta1, beta2, eps)
        losses.append(loss)
    return np.array(losses)
