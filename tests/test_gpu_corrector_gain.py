"""Gain of the learned corrector: trained on paired bounce-back /
immersed-boundary runs of six seeds, it must bring the near-surface
dissipation of a held-out seed closer to the bounce-back reference than the
plain immersed-boundary central difference does."""
import numpy as np
import pytest

import synth
from oracle import corrector as oc
from paper_1906_05448_amd import corrector, lbm
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu


def test_corrector_reduces_near_surface_dissipation_error():
    import torch
    cfg = corrector.PairConfig()
    nu = (cfg.tau - 0.5) / 3
    parts = [corrector.paired_samples(cfg, seed) for seed in range(6)]
    x = torch.cat([p[0] for p in parts])
    t = torch.cat([p[1] for p in parts])
    net = lbm.Mlp(synth.mlp_initial_params(0))
    losses = corrector.train(net, x, t, steps=4000, batch=4096, lr=1e-3, seed=0)
    assert losses[-100:].mean() < 0.5 * losses[:10].mean()
    xe, te, tbe = corrector.paired_samples(cfg, 7)
    y = net.forward(xe).cpu().numpy()[:, :9].astype(np.float64)
    plain = tbe.cpu().numpy()[:, :9].astype(np.float64)
    G_ref = (te.cpu().numpy()[:, :9].astype(np.float64) + plain) * cfg.u_rms
    G_ibm = plain * cfg.u_rms
    G_mlp = oc.corrected_gradient(plain, y, cfg.u_rms)
    e_ref = oc.dissipation_from_gradient(G_ref, nu)
    err_plain = rel_l2(oc.dissipation_from_gradient(G_ibm, nu), e_ref)
    err_mlp = rel_l2(oc.dissipation_from_gradient(G_mlp, nu), e_ref)
    print(f"samples {x.shape[0]} train, {xe.shape[0]} held out; loss {losses[:10].mean():.4f} -> "
          f"{losses[-100:].mean():.4f}; eps rel L2 vs bounce-back: plain IBM {err_plain:.3f}, corrected {err_mlp:.3f}")
    assert err_mlp < 0.6 * err_plain
    net.close()
