"""Parity of the warm-start network kernels with the FP64 reference."""
import numpy as np
import pytest
import torch

from oracle import adam as oadam
from oracle import cnn
from paper_2303_04679_amd.warmstart import NetConfig, WarmStartNet
from tests.gpu_helpers import need_gpu, rel

pytestmark = pytest.mark.gpu


def _net(size=64, batch=3, widths=(8, 12, 10)):
    cfg = NetConfig(batch=batch, size=size, n_obs=20, width1=widths[0], width2=widths[1],
                    width3=widths[2], out_ch=3)
    return cfg, WarmStartNet(cfg, seed=3)


def _inputs(cfg, seed):
    g = np.random.default_rng(seed)
    B, S = cfg.batch, cfg.size
    idx = np.stack([np.sort(g.choice(S * S, cfg.n_obs, replace=False)) for _ in range(B)]).astype(np.int32)
    u = g.normal(0, 0.3, (B, cfg.n_obs)).astype(np.float32)
    v = g.normal(0, 0.3, (B, cfg.n_obs)).astype(np.float32)
    re = g.uniform(100, 1000, B).astype(np.float32)
    return idx, u, v, re


def test_rasterize_and_forward():
    need_gpu()
    cfg, net = _net()
    idx, u, v, re = _inputs(cfg, 1)
    T = lambda a: torch.tensor(a, device="cuda")
    img = net.rasterize(T(idx), T(u), T(v), T(re))
    out = net.forward(cfg.batch)
    torch.cuda.synchronize()
    rimg = cnn.rasterize(cfg.size, idx, u, v, re.astype(np.float64), cfg.re_center, cfg.re_scale)
    np.testing.assert_allclose(img.cpu().numpy().reshape(rimg.shape), rimg, rtol=1e-6, atol=0)
    specs = cnn.layer_specs(cfg.width1, cfg.width2, cfg.width3, cfg.out_ch)
    th = cnn.bf16_round(net.master.cpu().numpy())
    ract, rout = cnn.forward(th, specs, img.cpu().double().numpy().reshape(rimg.shape))
    assert rel(out.cpu().numpy(), rout.numpy()) < 1e-5
    assert rel(net.acts[:cfg.batch].cpu().numpy(), ract.numpy()) < 1e-5
    # bf16 copy is the round-to-nearest-even of the masters
    bits = net.bf16.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    np.testing.assert_array_equal(bits.view(np.float32).astype(np.float64), th.numpy())


def test_loss_gradient_and_adam():
    need_gpu()
    cfg, net = _net()
    idx, u, v, re = _inputs(cfg, 2)
    T = lambda a: torch.tensor(a, device="cuda")
    img = net.rasterize(T(idx), T(u), T(v), T(re))
    net.forward(cfg.batch)
    tgt = torch.tensor(np.random.default_rng(4).normal(0, 0.2, (cfg.batch, int(net.lay.out_size))),
                       dtype=torch.float32, device="cuda")
    loss = net.loss_backward(cfg.batch, tgt)
    torch.cuda.synchronize()
    specs = cnn.layer_specs(cfg.width1, cfg.width2, cfg.width3, cfg.out_ch)
    th = cnn.bf16_round(net.master.cpu().numpy())
    rl, rg = cnn.loss_and_grad(th.numpy(), specs, img.cpu().double().numpy().reshape(cfg.batch, 4, cfg.size, cfg.size),
                               tgt.cpu().double().numpy())
    assert abs(float(loss) - rl) <= 1e-5 * rl
    assert rel(net.grad.cpu().numpy(), rg) < 1e-5
    w0 = net.master.cpu().numpy().astype(np.float64)
    g0 = net.grad.cpu().numpy().astype(np.float64)
    net.adam(1e-3)
    torch.cuda.synchronize()
    rw, _, _ = oadam.adam_step(w0, 0 * w0, 0 * w0, g0, 1e-3, 0.9, 0.999, 1e-8, 1)
    assert rel(net.master.cpu().numpy(), rw) < 1e-6
    bits = net.bf16.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    np.testing.assert_array_equal(bits.view(np.float32), cnn.bf16_round(net.master.cpu().numpy()).numpy().astype(np.float32))
