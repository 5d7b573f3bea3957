"""Writes the FP64 oracle's reference values for the 128^3 particle-laden
comparison (the production recipe of Sec. 3.1, Table 2 scaled to a 128^3
subset: decaying turbulence with E(k) ~ k^4 exp(-2 (k/4)^2), u_rms 0.03,
tau 0.52, 98 released spheres of radius 8, about 10% volume fraction,
density ratio 4), for bounce-back and for the immersed boundary
(r_d = 0.4), at steps 1, 10 and 100.

Stored per step: the velocity and density at 2048 seeded nodes with the
oracle's fluid flag there, every sphere's X, U, Omega, force and torque, the
snapshot statistics (Sec. 3.2) with 32 distance bins of width 1/4, and the
masked energy and dissipation spectra (Sec. 3.2.1).

Calls only the oracle and the seeded input generators:
    python tests/golden/make_particle_laden_128.py ibb
    python tests/golden/make_particle_laden_128.py ibm
(about 50 min of CPU each). Output: particle_laden_128_<bc>.npz here.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import stats as ostats  # noqa: E402
from oracle.sim import RELEASE, Config as OConfig, Sim as OSim  # noqa: E402

N = 128
N_SPHERES = 98
RADIUS = 8.0
RHO_P = 4.0
TAU = 0.52
U_RMS = 0.03
RD = 0.4
MIN_GAP = 2.0
STEPS = (1, 10, 100)
N_SAMPLES = 2048
NBINS, BIN_WIDTH = 32, 0.25
KMAX = 64


def inputs():
    """Seeded inputs shared with the GPU comparison: initial field, sphere
    centres, sampled node indices (flat, x fastest)."""
    spec = synth.hit_spectrum(seed=0, u_rms=U_RMS)
    u0 = synth.hit_field(spec, (N, N, N))
    X = synth.random_spheres(N_SPHERES, (N, N, N), 2 * RADIUS + MIN_GAP, seed=0)
    idx = np.random.default_rng(128).choice(N ** 3, size=N_SAMPLES, replace=False).astype(np.int64)
    return u0, X, np.sort(idx)


def main(bc):
    u0, X, idx = inputs()
    sim = OSim(OConfig(shape=(N, N, N), tau=TAU, bc=bc, ibm_retraction=RD))
    sim.set_fields(u0)
    sim.set_particles(X, r=np.full(N_SPHERES, RADIUS), rho_p=np.full(N_SPHERES, RHO_P), mode=RELEASE)
    nu = (TAU - 0.5) / 3.0
    out = {"idx": idx, "steps": np.array(STEPS)}
    done = 0
    t0 = time.time()
    for s in STEPS:
        sim.step(s - done)
        done = s
        u, rho = sim.fields()
        P = sim.state.P
        fluid = sim.fluid_mask().reshape(-1)
        F, T, Fc = sim.forces()
        st = ostats.statistics(u, rho, nu, (N, N, N), P.X, P.U, P.Om, P.r, P.rho, width=BIN_WIDTH, nbins=NBINS)
        owner, _ = ostats.classify((N, N, N), P.X, P.r, None, BIN_WIDTH, NBINS)
        um = ostats.masked_velocity(u, owner, P.X, P.U, P.Om, (N, N, N))
        k, E = ostats.energy_spectrum(um, KMAX)
        D = ostats.dissipation_spectrum(k, E, nu)
        p = f"s{s}_"
        out[p + "u"] = u.reshape(3, -1)[:, idx]
        out[p + "rho"] = rho.reshape(-1)[idx]
        out[p + "fluid"] = fluid[idx]
        out[p + "X"], out[p + "U"], out[p + "Om"] = P.X.copy(), P.U.copy(), P.Om.copy()
        out[p + "F"], out[p + "T"], out[p + "Fc"] = F, T, Fc
        for key in ("n_fluid", "mass", "ke_raw", "ke_masked", "ke_fluid", "eps_raw", "eps_masked", "eps_fluid",
                    "umax", "bulk_u"):
            out[p + "stat_" + key] = np.float64(st[key])
        out[p + "stat_momentum"] = st["momentum"]
        out[p + "hist"] = st["hist"][:5]
        out[p + "E"], out[p + "D"] = E, D
        print(f"{bc}: step {s} done after {time.time() - t0:.0f} s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"particle_laden_128_{bc}.npz")
    np.savez_compressed(path, **out)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
