"""The marching restriction kernel (T^T one axis at a time, Adam fused) against
the FP64 oracle's transpose of the decomposition and against the per-cell
gather kernel, on shapes that exercise every lane layout: rows of 16 and 32
coarse cells packed several to a wave, rows of exactly 64, rows split over
several 64-lane segments, 2-D fields, batches, and every tile option."""
import numpy as np
import pytest
import torch

from oracle import multigrid as mg
from oracle import operators as ops
from tests.gpu_helpers import (assert_levels, context_of, levels_of, need_gpu, pack_of, rel,
                               rounded)
from tests.oracle_cases import case, random_levels

pytestmark = pytest.mark.gpu

SHAPES = [
    ("poisson", (16, 32, 256), 3),   # coarse rows of 128: two 64-lane segments
    ("poisson", (32, 64, 64), 3),    # rows of 32 then 16: row groups share a wave
    ("poisson", (64, 128), 3),       # 2-D field, no z march
    ("cavity", (64, 64), 3),         # three 2-D fields
    ("ns3d", (32, 32, 64), 3),       # five 3-D fields, rows of 32 / 16
]


def _restrict_ref(ctx, spec, g, L):
    out = []
    for f, name in enumerate(spec.fields):
        axes = ops.field_axes(spec.op, name, spec.ndim)
        fine = torch.tensor(ctx.fine_views(g)[f].cpu().numpy())
        out.append([r.numpy() for r in mg.decompose_transpose(fine, L, axes)])
    return [[out[f][li] for f in range(len(spec.fields))] for li in range(L)]


@pytest.mark.parametrize("op,dims,L", SHAPES)
def test_restrict_matches_oracle_transpose(op, dims, L):
    need_gpu()
    spec = case(op, dims, L, seed=21)
    ctx = context_of(spec, "f64")
    gen = torch.Generator(device="cpu").manual_seed(22)
    g = torch.randn(int(ctx.lay.fine_total), generator=gen, dtype=torch.float64).cuda()
    pk = ctx.restrict_adjoint(g)
    ctx.set_march(False)
    pk2 = ctx.restrict_adjoint(g)
    torch.cuda.synchronize()
    ref = _restrict_ref(ctx, spec, g, L)
    assert_levels(levels_of(ctx, pk), ref, 1e-14, "march")
    assert rel(pk.cpu().numpy(), pk2.cpu().numpy()) <= 1e-14


@pytest.mark.parametrize("rows,planes", [(2, 1), (2, 2), (2, 4), (2, 8), (4, 1), (4, 2), (4, 4), (4, 8),
                                         (4, 16), (8, 4), (8, 8)])
def test_every_tile(rows, planes):
    need_gpu()
    spec = case("poisson", (32, 64, 128), 2, seed=23)
    ctx = context_of(spec, "f64")
    ctx.set_march_tile(rows, planes)
    gen = torch.Generator(device="cpu").manual_seed(24)
    g = torch.randn(int(ctx.lay.fine_total), generator=gen, dtype=torch.float64).cuda()
    pk = ctx.restrict_adjoint(g)
    torch.cuda.synchronize()
    assert_levels(levels_of(ctx, pk), _restrict_ref(ctx, spec, g, 2), 1e-14, (rows, planes))


def test_unsupported_tile_is_rejected():
    need_gpu()
    spec = case("poisson", (32, 32, 32), 2, seed=25)
    ctx = context_of(spec, "f64")
    with pytest.raises(Exception):
        ctx.set_march_tile(3, 1)
    with pytest.raises(Exception):
        ctx.set_march_tile(8, 1)


def test_batch_instances():
    need_gpu()
    spec = case("poisson", (32, 32, 64), 3, seed=26)
    ctx = context_of(spec, "f64", batch=3)
    gen = torch.Generator(device="cpu").manual_seed(27)
    g = torch.randn(int(ctx.lay.fine_total), generator=gen, dtype=torch.float64).cuda()
    pk = ctx.restrict_adjoint(g)
    torch.cuda.synchronize()
    for b in range(3):
        out = []
        fine = torch.tensor(ctx.fine_views(g, b)[0].cpu().numpy())
        ref = [[r.numpy()] for r in mg.decompose_transpose(fine, 3, (0, 1, 2))]
        assert_levels(levels_of(ctx, pk, b), ref, 1e-14, ("instance", b))


def test_step_march_equals_gather_f64():
    """The full iteration with Adam fused into the marching restriction equals
    the one with the gather kernel (up to the order of the sums)."""
    need_gpu()
    spec = case("ns3d", (32, 32, 64), 3, seed=28)
    lv = random_levels(spec, 29)
    outs = []
    for march in (True, False):
        ctx = context_of(spec, "f64")
        ctx.set_march(march)
        a = pack_of(ctx, [lv])
        b, m, v = ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
        for t in range(1, 4):
            ctx.step(a, b, m, v, t, lr=1e-2)
            a, b = b, a
        torch.cuda.synchronize()
        outs.append((a.cpu().numpy(), m.cpu().numpy(), v.cpu().numpy()))
    for x, y in zip(*outs):
        assert rel(x, y) <= 1e-12


def test_step_is_loss_grad_then_adam_f32_march():
    """FP32: the fused step (Adam inside the marching restriction) equals
    loss_grad (marching restriction alone) followed by the Adam kernel."""
    need_gpu()
    spec = case("ns3d", (32, 32, 64), 3, seed=30)
    lv = rounded(random_levels(spec, 31), "f32")
    ctx = context_of(spec, "f32")
    th = pack_of(ctx, [lv])
    out1, m1, v1 = ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    out2, m2, v2 = ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    ctx.step(th, out1, m1, v1, 1, lr=1e-2)
    _, g = ctx.loss_grad(th)
    ctx.adam(th, out2, m2, v2, g, 1, lr=1e-2)
    torch.cuda.synchronize()
    assert torch.equal(m1, m2) and torch.equal(v1, v2)
    assert rel(out1.cpu().numpy(), out2.cpu().numpy()) <= 1e-7


def test_restrict_f32_matches_oracle():
    """FP32 gradients on every level of a 64^3 channel problem against the FP64
    oracle, coarse levels held to the FP32 bound times their cancellation."""
    need_gpu()
    spec = case("ns3d", (64, 64, 64), 4, seed=32)
    lv = rounded(random_levels(spec, 33), "f32")
    ctx = context_of(spec, "f32")
    th = pack_of(ctx, [lv])
    _, g = ctx.loss_grad(th)
    torch.cuda.synchronize()
    _, rgrad = ops.loss_and_grad(spec, lv)
    assert_levels(levels_of(ctx, g), rgrad, 1e-5, "f32", spec=spec)


@pytest.mark.parametrize("op,dims,L,batch", [("poisson", (200,), 4, 1), ("heat", (64, 32), 4, 2),
                                             ("poisson_node", (32, 32), 4, 2),
                                             ("cavity", (64, 64), 4, 3), ("ns3d", (32, 32, 32), 4, 1),
                                             ("burgers", (64, 64), 5, 1)])
def test_lds_tail_equals_per_level_launches(op, dims, L, batch):
    """The one-launch LDS tail (small levels of each instance in one block)
    gives the per-level kernels' prolongation, gradient and Adam state."""
    need_gpu()
    spec = case(op, dims, L, seed=34)
    lvs = [random_levels(spec, 35 + b, lo=0.05, hi=0.6) for b in range(batch)]
    outs = []
    for tail in (True, False):
        ctx = context_of(spec, "f64", batch=batch)
        ctx.set_tail(tail)
        a = pack_of(ctx, lvs)
        fine = ctx.prolong(a)
        b, m, v = ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
        for t in range(1, 3):
            ctx.step(a, b, m, v, t, lr=1e-2)
            a, b = b, a
        _, g = ctx.loss_grad(a)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy() for x in (fine, a, m, v, g)])
    for x, y in zip(*outs):
        assert rel(x, y) <= 1e-13


@pytest.mark.parametrize("op,dims,L", SHAPES + [("poisson", (16, 8, 64), 3), ("heat", (64, 32), 3)])
def test_block_prolongation_matches_oracle(op, dims, L):
    """The block Horner step (one coarse cell per thread, x neighbours by
    shuffles) against the oracle's decomposition and the per-cell kernel."""
    need_gpu()
    spec = case(op, dims, L, seed=36)
    lv = random_levels(spec, 37)
    ctx = context_of(spec, "f64")
    theta = pack_of(ctx, [lv])
    fine = ctx.prolong(theta)
    ctx.set_march(False)
    fine2 = ctx.prolong(theta)
    torch.cuda.synchronize()
    for f, name in enumerate(spec.fields):
        axes = ops.field_axes(spec.op, name, spec.ndim)
        ref = mg.decompose_horner([torch.tensor(r[f]) for r in lv], axes).numpy()
        assert rel(ctx.fine_views(fine)[f].cpu().numpy(), ref) <= 1e-14
    assert rel(fine.cpu().numpy(), fine2.cpu().numpy()) <= 1e-14
