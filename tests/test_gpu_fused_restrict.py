"""MODIL_FLAG_FUSED_RESTRICT: the fused channel-flow kernel sums the finest
gradient over the fine planes of each level-1 plane (z part of M_L^T) and the
assembly kernel applies T^T in y and x, adds the sums of neighbouring
z-chunks and updates level 1.  Checked against the oracle and against the
default path (finest gradient written, then restricted), over z-chunks of 2,
4, 8 and 16 planes, ragged xy tiles, two to four levels."""
import numpy as np
import pytest
import torch

from oracle import operators as ops
from paper_2303_04679_amd import configs, synth
from paper_2303_04679_amd.modil import Context
from tests.gpu_helpers import (TERMS, TOL, assert_levels, assert_terms, levels_of, need_gpu, pack_of,
                               problem_of, rounded)
from tests.oracle_cases import case, random_levels
from tests.workload_oracle import oracle_spec

pytestmark = pytest.mark.gpu


def _ctx(spec, batch=1, specs=None, restrict=True):
    specs = specs or [spec] * batch
    prob = problem_of(spec, "f32", batch)
    prob.fused_restrict = restrict
    ctx = Context(prob)
    for b, s in enumerate(specs):
        for field, term, idx, vals, w in s.meas:
            ctx.set_measurements(field, idx, vals, w, term=term, instance=b)
    for e in range(4):
        if e in spec.forcing:
            arr = np.stack([np.asarray(s.forcing[e]).ravel() for s in specs])
            ctx.set_field(f"forcing{e}", torch.tensor(arr, dtype=ctx.dtype, device="cuda").reshape(-1))
    if spec.op == "ns3d_fixed":
        arr = np.stack([np.asarray(s.chi).ravel() for s in specs])
        ctx.set_field("chi", torch.tensor(arr, dtype=ctx.dtype, device="cuda").reshape(-1))
    return ctx


@pytest.mark.parametrize("op,dims,L", [("ns3d", (24, 36, 60), 3), ("ns3d_fixed", (16, 28, 24), 3),
                                       ("ns3d", (64, 16, 32), 4), ("ns3d", (16, 16, 24), 2),
                                       ("ns3d", (32, 32, 64), 4)])
def test_fused_restrict_matches_oracle_and_default(op, dims, L):
    need_gpu()
    print(f"\n[fused-restrict] {op} {dims} L={L}", flush=True)
    spec = case(op, dims, L, seed=13, with_forcing=True)
    lv = rounded(random_levels(spec, 14), "f32")
    rterms, rgrad = ops.loss_and_grad(spec, lv)
    ctx = _ctx(spec)
    assert ctx.fused_active()
    theta = pack_of(ctx, [lv])
    tf, gf = ctx.loss_grad(theta)
    ref = _ctx(spec, restrict=False)
    td, gd = ref.loss_grad(pack_of(ref, [lv]))
    torch.cuda.synchronize()
    assert_terms(tf[0].cpu().numpy(), rterms, TOL["f32"], "fused restrict")
    assert_levels(levels_of(ctx, gf), rgrad, TOL["f32"], "fused restrict", spec=spec)
    assert_levels(levels_of(ctx, gf), levels_of(ref, gd), TOL["f32"], "vs default", spec=spec)
    # one full step from zero moments: m = (1 - b1) g on every level
    out, m, v = ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    ctx.step(theta, out, m, v, 1, lr=1e-2)
    torch.cuda.synchronize()
    assert_levels(levels_of(ctx, m), [[0.1 * g for g in row] for row in rgrad], TOL["f32"], "m", spec=spec)


@pytest.mark.parametrize("batch", [4, 26, 52, 86])
def test_fused_restrict_zchunks(batch):
    """z-chunks of 2, 4, 8 and 16 planes (the batch sizes select them), 40
    planes so that the longer chunks end ragged."""
    need_gpu()
    dims = (40, 12, 20)
    print(f"\n[fused-restrict] z-chunks {dims} batch={batch}", flush=True)
    specs = [case("ns3d", dims, 3, seed=300 + b) for b in range(batch)]
    ctx = _ctx(specs[0], batch=batch, specs=specs)
    ref = _ctx(specs[0], batch=batch, specs=specs, restrict=False)
    lvs = [rounded(random_levels(s, 400 + b), "f32") for b, s in enumerate(specs)]
    tf, gf = ctx.loss_grad(pack_of(ctx, lvs))
    tg, gg = ref.loss_grad(pack_of(ref, lvs))
    torch.cuda.synchronize()
    for b in range(batch):
        assert_terms(tf[b].cpu().numpy(), {t: float(tg[b, k]) for k, t in enumerate(TERMS)}, TOL["f32"], b)
        assert_levels(levels_of(ctx, gf, b), levels_of(ref, gg, b), TOL["f32"], b, spec=specs[b])
    for b in (0, batch - 1):
        rt, rg = ops.loss_and_grad(specs[b], lvs[b])
        assert_levels(levels_of(ctx, gf, b), rg, TOL["f32"], ("oracle", b), spec=specs[b])


def test_fused_restrict_run_equals_steps():
    need_gpu()
    spec = case("ns3d", (32, 32, 64), 4, seed=21, with_forcing=True)
    lv = rounded(random_levels(spec, 22), "f32")
    ctx = _ctx(spec)
    th0 = pack_of(ctx, [lv])
    a, b, m, v = th0.clone(), ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    res = ctx.run(a, b, m, v, 3, 4, lr=1e-3)
    a2, b2, m2, v2 = th0.clone(), ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    for k in range(4):
        ctx.step(a2, b2, m2, v2, 3 + k, lr=1e-3)
        a2, b2 = b2, a2
    torch.cuda.synchronize()
    assert torch.equal(res, a2) and torch.equal(m, m2) and torch.equal(v, v2)


def test_fused_restrict_workload_ns3d128():
    need_gpu()
    wl = configs.WORKLOADS["ns3d128"]()
    wl.spec.fused_restrict = True
    ctx, theta0 = configs.build(wl)
    spec = oracle_spec(wl)
    shapes = ops.level_shapes(spec.op, spec.dims, spec.n_levels, spec.centering)
    lv = synth.uniform_levels(shapes, 90, -0.5, 0.5)
    base = [[v.detach().cpu().double().numpy() for v in row] for row in ctx.level_views(theta0)]
    lv = rounded([[b + x for b, x in zip(br, xr)] for br, xr in zip(base, lv)], "f32")
    terms, grad = ctx.loss_grad(pack_of(ctx, [lv]))
    torch.cuda.synchronize()
    rterms, rgrad = ops.loss_and_grad(spec, lv)
    assert_terms(terms[0].cpu().numpy(), rterms, TOL["f32"], "ns3d128")
    assert_levels(levels_of(ctx, grad), rgrad, TOL["f32"], "ns3d128", spec=spec)
