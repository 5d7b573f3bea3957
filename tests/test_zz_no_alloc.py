"""The network gradient without allocation (lbm_mlp_gradient_noalloc), for
callers that cannot allocate device memory: called through the C ABI twice
in a row, the second time on fewer samples, it matches lbm_mlp_gradient on
the same inputs bit for bit (same kernels, partial sums in the library's
per-device scratch array instead of the network's workspace)."""
import numpy as np
import pytest

import synth
from paper_1906_05448_amd import lbm

pytestmark = pytest.mark.gpu


def _inputs(torch, n, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((n, lbm.MLP_IN_STRIDE), np.float32)
    x[:, :lbm.MLP_IN] = rng.normal(size=(n, lbm.MLP_IN))
    t = np.zeros((n, lbm.MLP_OUT_STRIDE), np.float32)
    t[:, :lbm.MLP_OUT] = rng.normal(scale=0.3, size=(n, lbm.MLP_OUT))
    return (torch.from_numpy(x).to(torch.bfloat16).cuda().contiguous(), torch.from_numpy(t).cuda().contiguous())


def test_gradient_noalloc_matches_gradient():
    import torch
    net = lbm.Mlp(synth.mlp_initial_params(3))
    grad = torch.full((lbm.MLP_PARAMS,), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    for n, seed in ((70000, 1), (1500, 2)):
        x, t = _inputs(torch, n, seed)
        net.gradient_noalloc(x, t, grad, loss)
        net.sync()
        g_static = grad.cpu().numpy().copy()
        l_static = float(loss.cpu().numpy()[0])
        l_ref, g_ref = net.gradient(x, t, want_grad=True)
        assert np.isfinite(g_static).all()
        assert np.array_equal(g_static, g_ref), n
        assert l_static / (9.0 * n) == l_ref, n
    # argument checks reject before any work
    with pytest.raises(lbm.LbmError) as e:
        lbm._check(lbm.lib().lbm_mlp_gradient_noalloc(None, None, None, 10, None, None, None), "noalloc")
    assert e.value.status == -1
    x, t = _inputs(torch, 8, 3)
    with pytest.raises(lbm.LbmError) as e:
        lbm._check(lbm.lib().lbm_mlp_gradient_noalloc(lbm.lib().lbm_mlp_device_params(net._h), lbm._dev(x),
                                                      lbm._dev(t), (1 << 30) + 1, lbm._dev(grad), lbm._dev(loss),
                                                      None), "noalloc")
    assert e.value.status == -3
    net.close()
