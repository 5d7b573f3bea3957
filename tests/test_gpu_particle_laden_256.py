"""The 256^3 particle-laden case (Sec. 3.1, Table 2 recipe): decaying
turbulence with E(k) ~ k^4 exp(-2 (k/4)^2), u_rms 0.03, tau 0.52, 780 freely
moving spheres of radius 8 (about 10% volume fraction), FP16 shifted storage
with FP32 collision, bounce-back and immersed boundary, 5000 steps.

At this size the FP64 oracle is out of reach, so the checks are ones that
hold at any size: the FP16 run follows the FP32 run (which itself matches
the oracle at 1e-5 in the smaller parity tests) to the FP16 bar while the
flow is still deterministic at this precision (100 steps), the runs stay
finite and overlap-free for all 5000 steps, fluid mass is conserved, and the
kinetic energy and dissipation histories of the two precisions agree while
the field itself decorrelates."""
import numpy as np
import pytest

import synth
from paper_1906_05448_amd import lbm
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu

N = 256
N_SPHERES = 780
RADIUS = 8.0
TAU = 0.52


def _lattice(bc, store, rho_p, u0, X):
    lat = lbm.Lattice(lbm.Config(nx=N, ny=N, nz=N, tau=TAU, store=store, bc=bc, ibm_retraction=0.4,
                                 max_particles=N_SPHERES, max_radius=RADIUS))
    lat.set_fields(u0)
    lat.set_particles(X, RADIUS, rho_p=rho_p, mode=lbm.RELEASE, motion=lbm.MOTION_FREE)
    return lat


# Bounce-back at the configuration's neutral buoyancy; the immersed boundary
# at density ratio 4, the lightest at which its explicit inner-inertia
# coupling is stable for r = 8.
@pytest.mark.parametrize("bc,rho_p", [(lbm.BC_IBB, 1.0), (lbm.BC_IBM, 4.0)])
def test_256_cubed_780_spheres_fp16_follows_fp32(bc, rho_p):
    spec = synth.hit_spectrum(seed=3, u_rms=0.03)
    u0 = synth.hit_field(spec, (N, N, N), dtype=np.float32)
    X = synth.random_spheres(N_SPHERES, (N, N, N), 2 * RADIUS + 2.0, seed=3)
    runs = {s: _lattice(bc, s, rho_p, u0, X) for s in (lbm.STORE_F32, lbm.STORE_F16S)}
    a, b = runs[lbm.STORE_F32], runs[lbm.STORE_F16S]
    hist = {s: [] for s in runs}
    done = 0
    for target in (100, 1000, 2000, 3000, 4000, 5000):
        for lat in runs.values():
            lat.step(target - done)
        done = target
        for s, lat in runs.items():
            st = lat.stats(nbins=0)
            hist[s].append((st["mass"], st["ke_fluid"], st["eps_fluid"], st["n_fluid"]))
            assert np.isfinite(st["ke_fluid"]) and np.isfinite(st["eps_fluid"])
        if target == 100:
            ua, _ = a.get_fields()
            ub, _ = b.get_fields()
            fluid = np.isfinite(ua).all(0) & np.isfinite(ub).all(0)
            du = rel_l2(ub, ua, fluid)
            Fa, _, _ = a.forces()
            Fb, _, _ = b.forces()
            Xa, Ua, _ = a.get_particles()
            Xb, Ub, _ = b.get_particles()
            print(f"step 100: FP16 vs FP32 u rel L2 {du:.2e}, F rel L2 {rel_l2(Fb, Fa):.2e}, "
                  f"U rel L2 {rel_l2(Ub, Ua):.2e}, max |dX| {np.abs(Xb - Xa).max():.2e}", flush=True)
            assert du < 2e-3
            assert rel_l2(Fb, Fa) < 2e-2
            assert rel_l2(Ub, Ua) < 1e-2
    h32, h16 = np.array(hist[lbm.STORE_F32]), np.array(hist[lbm.STORE_F16S])
    for row32, row16, t in zip(h32, h16, (100, 1000, 2000, 3000, 4000, 5000)):
        print(f"step {t}: ke {row32[1]:.4e} / {row16[1]:.4e}, eps {row32[2]:.4e} / {row16[2]:.4e}, "
              f"mass/N_f {row32[0] / row32[3]:.8f} / {row16[0] / row16[3]:.8f}", flush=True)
    # energy decays; the two precisions keep the same history
    assert h32[-1, 1] < 0.8 * h32[0, 1]
    assert np.all(np.abs(h16[:, 1] / h32[:, 1] - 1) < 2e-2)
    assert np.all(np.abs(h16[:, 2] / h32[:, 2] - 1) < 5e-2)
    for s, lat in runs.items():
        Xs, _, _ = lat.get_particles()
        assert np.isfinite(Xs).all()
        lat.close()
