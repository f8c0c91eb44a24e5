"""The differentiable-loss pattern: torch.autograd.Function over the HIP adjoint.

Checks the gradient against central finite differences of the GPU loss on an
8^3 grid, against the PyTorch-autograd oracle on a 32^3 grid, and that torch
optimisers driven by it reproduce the library's fused step.
"""
import numpy as np
import pytest
import torch

from oracle import operators as ops
from paper_2303_04679_amd.autograd import modil_loss
from tests.gpu_helpers import (assert_levels, context_of, levels_of, need_gpu, pack_of, rel,
                               rounded)
from tests.oracle_cases import case, random_levels

pytestmark = pytest.mark.gpu


def test_gradient_matches_central_differences_8cube():
    need_gpu()
    spec = case("ns3d", (8, 8, 8), 2, seed=61)
    ctx = context_of(spec, "f64")
    theta = pack_of(ctx, [random_levels(spec, 62)]).requires_grad_(True)
    loss = modil_loss(theta, ctx)
    loss.backward()
    g = theta.grad.detach().clone()
    th = theta.detach().clone()
    n = th.numel()
    fd = torch.empty(n, dtype=torch.float64, device="cuda")
    for k in range(n):
        x0 = float(th[k])
        step = 1e-6 * max(1.0, abs(x0))
        th[k] = x0 + step
        lp = ctx.loss(th).sum()
        th[k] = x0 - step
        lm = ctx.loss(th).sum()
        th[k] = x0
        fd[k] = (lp - lm) / (2 * step)
    torch.cuda.synchronize()
    err = float(torch.linalg.norm(g - fd) / torch.linalg.norm(fd))
    assert err < 1e-6, err


def test_gradient_matches_torch_autograd_reference_32cube():
    """FP32 fields, FP64 loss: the autograd.Function gradient against the FP64
    PyTorch-autograd oracle on the same (FP32-rounded) inputs."""
    need_gpu()
    spec = case("ns3d", (32, 32, 32), 3, seed=63)
    lv = rounded(random_levels(spec, 64), "f32")
    ctx = context_of(spec, "f32")
    theta = pack_of(ctx, [lv]).requires_grad_(True)
    loss = modil_loss(theta, ctx)
    loss.backward()
    torch.cuda.synchronize()
    rterms, rgrad = ops.loss_and_grad(spec, lv)
    assert abs(float(loss) - sum(rterms.values())) <= 1e-5 * sum(rterms.values())
    assert_levels(levels_of(ctx, theta.grad), rgrad, 1e-5, "autograd")


def test_forward_keeps_no_fine_field():
    """The forward pass stores nothing beyond the parameter pack it was given."""
    need_gpu()
    spec = case("ns3d", (32, 32, 32), 3, seed=65)
    ctx = context_of(spec, "f32")
    theta = pack_of(ctx, [random_levels(spec, 66)]).requires_grad_(True)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    loss = modil_loss(theta, ctx)
    torch.cuda.synchronize()
    grown = torch.cuda.memory_allocated() - before
    fine_bytes = ctx.lay.fine_total * 4
    assert grown < fine_bytes // 100, (grown, fine_bytes)
    loss.backward()
    assert theta.grad is not None


def test_torch_optimiser_reproduces_fused_step():
    """torch.optim.Adam on the autograd gradient = modil_step (FP64)."""
    need_gpu()
    spec = case("ns3d", (16, 16, 16), 3, seed=67)
    lv = random_levels(spec, 68)
    ctx = context_of(spec, "f64")
    theta = pack_of(ctx, [lv]).requires_grad_(True)
    opt = torch.optim.Adam([theta], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    a = pack_of(ctx, [lv])
    b, m, v = ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    for t in range(1, 4):
        opt.zero_grad()
        modil_loss(theta, ctx).backward()
        opt.step()
        ctx.step(a, b, m, v, t, lr=1e-2)
        a, b = b, a
    torch.cuda.synchronize()
    assert rel(theta.detach().cpu().numpy(), a.cpu().numpy()) < 1e-12
