"""Parity of the matrix-core corrector network (BF16 operands, FP32
accumulation) with the FP64 reference: forward pass, gradient, Adam."""
import numpy as np
import pytest

import synth
from oracle import mlp as om
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _features(n, seed, scale=1.0):
    """Random features rounded to BF16: (device bf16 [n, 96], host FP64 [n, 85])."""
    torch = _torch()
    x = np.zeros((n, 96), np.float32)
    x[:, :85] = np.random.default_rng(seed).normal(size=(n, 85)) * scale
    xb = torch.from_numpy(x).to(torch.bfloat16)
    return xb.cuda().contiguous(), xb.float().numpy()[:, :85].astype(np.float64)


def _targets(n, seed):
    torch = _torch()
    t = np.zeros((n, 16), np.float32)
    t[:, :9] = np.random.default_rng(seed).normal(size=(n, 9)) * 0.5
    return torch.from_numpy(t).cuda(), t[:, :9].astype(np.float64)


def _params(seed, noise=0.05):
    th = synth.mlp_initial_params(seed)
    # perturbed (non-zero biases), exactly representable in FP32
    return (th + np.random.default_rng(seed + 100).normal(0, noise, om.N_PARAMS)).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000])
def test_forward_matches_reference(n):
    from paper_1906_05448_amd import lbm
    th = _params(1)
    net = lbm.Mlp(th)
    xd, xh = _features(n, 2)
    y = net.forward(xd).cpu().numpy()
    ref, _ = om.forward(th, xh)
    assert rel_l2(y[:, :9], ref) < 1e-2
    assert np.all(y[:, 9:] == 0.0)
    net.close()


def test_zero_weights_give_bias_and_large_batch():
    from paper_1906_05448_amd import lbm
    th = np.zeros(om.N_PARAMS)
    th[-9:] = np.linspace(-0.4, 0.4, 9)
    net = lbm.Mlp(th)
    xd, _ = _features(130, 3)
    y = net.forward(xd).cpu().numpy()
    assert np.array_equal(y[:, :9], np.broadcast_to(th[-9:].astype(np.float32), (130, 9)))
    # more samples than one pass of the grid: sampled rows against the reference
    th = _params(4)
    net.set_params(th)
    n = 300_001
    xd, xh = _features(n, 5)
    y = net.forward(xd).cpu().numpy()
    rows = np.r_[0:200, n - 200:n, np.random.default_rng(6).integers(0, n, 2000)]
    ref, _ = om.forward(th, xh[rows])
    assert rel_l2(y[rows, :9], ref) < 1e-2
    net.close()


@pytest.mark.parametrize("n", [1, 64, 777, 4096])
def test_gradient_matches_reference(n):
    from paper_1906_05448_amd import lbm
    th = _params(7)
    net = lbm.Mlp(th)
    xd, xh = _features(n, 8)
    td, th_t = _targets(n, 9)
    loss, g = net.gradient(xd, td, want_grad=True)
    L, gref = om.grad(th, xh, th_t)
    assert abs(loss - L) < 2e-2 * L
    assert rel_l2(g, gref) < 1e-2
    # per block: weights and biases of every layer
    offs = [0, 5440, 5504, 9600, 9664, 10240, 10249]
    for a, b in zip(offs[:-1], offs[1:]):
        assert rel_l2(g[a:b], gref[a:b]) < 2e-2, (a, b)
    net.close()


def test_adam_training_tracks_reference():
    from paper_1906_05448_amd import lbm
    th0 = _params(10, noise=0.0)
    net = lbm.Mlp(th0)
    n = 2048
    xd, xh = _features(n, 11, scale=0.7)
    t = np.zeros((n, 16), np.float32)
    t[:, :9] = np.tanh(xh[:, :9] * 0.8)
    td = _torch().from_numpy(t).cuda()
    th, m, v = th0.copy(), np.zeros(om.N_PARAMS), np.zeros(om.N_PARAMS)
    lg, lr_ = [], []
    for step in range(1, 31):
        l_gpu, _ = net.gradient(xd, td)
        net.adam_step(lr=3e-3)
        L, gg = om.grad(th, xh, t[:, :9].astype(np.float64))
        th, m, v = om.adam_step(th, gg, m, v, step, lr=3e-3)
        lg.append(l_gpu)
        lr_.append(L)
    lg, lr_ = np.array(lg), np.array(lr_)
    assert lg[-1] < 0.5 * lg[0]
    assert np.abs(lg - lr_).max() < 3e-2 * lr_[0]
    pg = net.params().astype(np.float64)
    assert rel_l2(pg - th0, th - th0) < 0.1
    net.close()


def test_mlp_argument_errors():
    from paper_1906_05448_amd import lbm
    net = lbm.Mlp(np.zeros(om.N_PARAMS))
    with pytest.raises(lbm.LbmError):
        net.adam_step()  # no gradient yet
    xd, _ = _features(0, 1)
    assert net.forward(xd).shape == (0, 16)
    td = _torch().zeros((0, 16), dtype=_torch().float32, device="cuda")
    with pytest.raises(lbm.LbmError):
        net.gradient(xd, td)
    with pytest.raises(lbm.LbmError):
        net.adam_step(lr=-1.0)
    net.close()
