"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: norm-wise relative error per (level, field) and relative error
per loss term, 1e-12 in FP64 and 1e-5 in FP32 (FP32 inputs are promoted to
FP64 for the oracle).  Sizes span many 256-thread blocks with ragged tails
and non-square grids.
"""
import math

import numpy as np
import pytest
import torch

from oracle import adam as oadam
from oracle import multigrid as mg
from oracle import operators as ops
from tests.gpu_helpers import (TERMS, TOL, assert_levels, assert_terms, context_of, levels_of, need_gpu,
                               pack_of, rel, rounded)
from tests.oracle_cases import case, random_levels

pytestmark = pytest.mark.gpu

CASES = [
    ("poisson", (200,), 4),
    ("poisson", (32, 48), 4),
    ("poisson", (16, 8, 24), 3),
    ("burgers", (64, 64), 5),
    ("burgers", (24, 40), 3),
    ("heat", (64, 32), 4),
    ("heat", (40, 72), 3),
    ("heat", (128, 64), 4),
    ("heat", (96, 96), 3),
    ("ns3d", (16, 16, 24), 3),
    ("ns3d_fixed", (8, 16, 24), 3),
    ("cavity", (32, 48), 4),
    ("poisson_node", (64,), 4),
    ("poisson_node", (16, 24), 3),
    ("poisson_node", (8, 16, 8), 2),
    ("cavity_node", (32, 48), 4),
    ("cavity_node", (24, 16), 3),
    ("ns3d_node", (16, 16, 24), 3),
    ("ns3d_node", (8, 12, 20), 2),
    ("ns3d_fixed_node", (8, 16, 24), 3),
]


def _levels(spec, seed):
    if spec.op == "burgers":
        return random_levels(spec, seed, lo=0.05, hi=0.6)
    return random_levels(spec, seed)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("op,dims,L", CASES)
def test_loss_grad(op, dims, L, dtype):
    need_gpu()
    print(f"\n[parity] loss_grad {op} {dims} L={L} {dtype}", flush=True)
    spec = case(op, dims, L, seed=7, with_forcing=op != "poisson")
    lv = rounded(_levels(spec, 8), dtype)
    ref_terms, ref_grad = ops.loss_and_grad(spec, lv)
    ctx = context_of(spec, dtype)
    theta = pack_of(ctx, [lv])
    terms, grad = ctx.loss_grad(theta)
    terms2 = ctx.loss(theta)
    torch.cuda.synchronize()
    tol = TOL[dtype]
    assert_terms(terms[0].cpu().numpy(), ref_terms, tol, op)
    assert_terms(terms2[0].cpu().numpy(), ref_terms, tol, op)
    assert_levels(levels_of(ctx, grad), ref_grad, tol, op)


@pytest.mark.parametrize("op,dims,L", [("poisson", (48, 32), 4), ("heat", (32, 64), 4),
                                       ("ns3d", (8, 16, 8), 3), ("poisson_node", (48, 32), 4),
                                       ("poisson_node", (16, 8, 16), 3),
                                       ("poisson", (16, 512), 3), ("poisson", (4, 8, 256), 2)])
def test_prolong_and_restrict(op, dims, L):
    """Horner prolongation and M_L^T against the oracle.  The last two shapes
    have coarse rows of 128 and 256 cells, which the block prolongation and
    the marching restriction take in several 64-lane segments."""
    need_gpu()
    spec = case(op, dims, L, seed=1)
    lv = _levels(spec, 2)
    ctx = context_of(spec, "f64")
    theta = pack_of(ctx, [lv])
    fine = ctx.prolong(theta)
    torch.cuda.synchronize()
    for f, name in enumerate(spec.fields):
        axes = ops.field_axes(spec.op, name, spec.ndim)
        ref = mg.decompose_horner([torch.tensor(r[f]) for r in lv], axes, spec.centering).numpy()
        got = ctx.fine_views(fine)[f].cpu().numpy()
        assert rel(got, ref) <= 1e-14
    g = torch.randn(fine.numel(), dtype=torch.float64, device="cuda")
    pk = ctx.restrict_adjoint(g)
    torch.cuda.synchronize()
    gl = levels_of(ctx, pk)
    for f, name in enumerate(spec.fields):
        axes = ops.field_axes(spec.op, name, spec.ndim)
        ref = mg.decompose_transpose(torch.tensor(ctx.fine_views(g)[f].cpu().numpy()), L, axes,
                                     spec.centering)
        for li in range(L):
            assert rel(gl[li][f], ref[li].numpy()) <= 1e-14


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adam(dtype):
    need_gpu()
    spec = case("cavity", (32, 32), 3, seed=2)
    ctx = context_of(spec, dtype)
    rng = np.random.default_rng(5)
    n = int(ctx.lay.total)
    th = rng.standard_normal(n)
    m = 0.1 * rng.standard_normal(n)
    v = np.abs(rng.standard_normal(n))
    g = rng.standard_normal(n)
    T = lambda a: torch.tensor(a, dtype=ctx.dtype, device="cuda")
    cast = (lambda a: a) if dtype == "f64" else (lambda a: a.astype(np.float32).astype(np.float64))
    th_t, th_o, m_t, v_t, g_t = T(th), T(th) * 0, T(m), T(v), T(g)
    ctx.adam(th_t, th_o, m_t, v_t, g_t, step=7, lr=1e-2)
    torch.cuda.synchronize()
    rt, rm, rv = oadam.adam_step(cast(th), cast(m), cast(v), cast(g), 1e-2, 0.9, 0.999, 1e-8, 7)
    tol = 1e-14 if dtype == "f64" else 1e-6
    assert rel(th_o.cpu().numpy(), rt) <= tol
    assert rel(m_t.cpu().numpy(), rm) <= tol
    assert rel(v_t.cpu().numpy(), rv) <= tol


@pytest.mark.parametrize("op,dims,L", [("burgers", (32, 32), 4), ("heat", (32, 32), 4),
                                       ("ns3d", (8, 8, 16), 3), ("cavity", (32, 32), 4),
                                       ("poisson_node", (32, 32), 4), ("cavity_node", (32, 32), 4),
                                       ("ns3d_node", (8, 8, 16), 3), ("ns3d", (32, 32, 64), 4),
                                       ("heat", (128, 64), 4), ("heat", (96, 96), 3)])
def test_step_sequence_f64(op, dims, L):
    """Three modil_step calls (ping-pong theta) follow the oracle's loss, gradient and Adam.
    The 32 x 32 x 64 channel starts its restriction tail at a level of 8192
    cells (copied into LDS in rounds of eight loads per thread) and updates
    three levels there.  On the 128 x 64 heat grid the marching kernel
    restricts u alone from the finest level while the tail takes the 1-D q
    from the finest level on, its column sums included; on the 96 x 96 grid
    the tail starts at level 1 and the column sums take their own launch."""
    need_gpu()
    spec = case(op, dims, L, seed=3)
    lv = _levels(spec, 4)
    ctx = context_of(spec, "f64")
    a, b = pack_of(ctx, [lv]), ctx.new_pack()
    m, v = ctx.new_pack(), ctx.new_pack()
    ref = [[(x.copy(), np.zeros_like(x), np.zeros_like(x)) for x in row] for row in lv]
    terms = torch.empty((1, 5), dtype=torch.float64, device="cuda")
    for t in range(1, 4):
        ctx.step(a, b, m, v, t, lr=1e-2, terms=terms)
        torch.cuda.synchronize()
        cur = [[s[0] for s in row] for row in ref]
        rterms, rgrad = ops.loss_and_grad(spec, cur)
        print(f"[parity] step {t} terms", {k: abs(float(terms[0, i]) - rterms[k]) / max(abs(rterms[k]), 1e-300)
                                            for i, k in enumerate(TERMS) if rterms[k]}, flush=True)
        assert_terms(terms[0].cpu().numpy(), rterms, 1e-12, (op, t))
        ref = [[oadam.adam_step(s[0], s[1], s[2], g, 1e-2, 0.9, 0.999, 1e-8, t)
                for s, g in zip(row, grow)] for row, grow in zip(ref, rgrad)]
        a, b = b, a
    for name, pk, k in (("theta", a, 0), ("m", m, 1), ("v", v, 2)):
        got, want = levels_of(ctx, pk), [[s[k] for s in row] for row in ref]
        print(f"[parity] {name}", max(rel(g, r) for gr, rr in zip(got, want) for g, r in zip(gr, rr)), flush=True)
        assert_levels(got, want, 1e-12, (op, name))


def test_burgers_zero_face_speed():
    """FP64 Burgers with faces of exactly zero speed: a finest level
    antisymmetric in x (coarse levels zero) gives u_{N/2-1} = -u_{N/2} in
    every row, so the middle face has (a + b)/2 = 0 and the upwind flux is at
    its kink.  The derivative of |s| at s = 0 is taken as 0 on both sides."""
    need_gpu()
    dims = (24, 40)
    spec = case("burgers", dims, 3, seed=9, with_forcing=True)
    lv = [[np.zeros(s) for s in row] for row in ops.level_shapes("burgers", dims, 3)]
    half = np.random.default_rng(31).uniform(0.05, 0.6, size=(dims[0], dims[1] // 2))
    lv[0][0] = np.concatenate([-half[:, ::-1], half], axis=1)
    fine = lv[0][0]
    assert np.all(fine[:, dims[1] // 2 - 1] + fine[:, dims[1] // 2] == 0.0)
    rterms, rgrad = ops.loss_and_grad(spec, lv)
    ctx = context_of(spec, "f64")
    terms, grad = ctx.loss_grad(pack_of(ctx, [lv]))
    torch.cuda.synchronize()
    assert_terms(terms[0].cpu().numpy(), rterms, 1e-12, "burgers kink")
    assert_levels(levels_of(ctx, grad), rgrad, 1e-12, "burgers kink")


@pytest.mark.parametrize("op,dims,L", [("heat", (32, 32), 4), ("ns3d", (8, 8, 16), 3)])
def test_step_is_loss_grad_then_adam_f32(op, dims, L):
    """In FP32 the fused step equals loss_grad followed by adam, bit for bit, and
    its loss terms match the oracle.  (Adam's first steps are sign-like, so an
    elementwise FP32 trajectory comparison is not meaningful.)"""
    need_gpu()
    spec = case(op, dims, L, seed=3)
    lv = rounded(_levels(spec, 4), "f32")
    ctx = context_of(spec, "f32")
    th = pack_of(ctx, [lv])
    out1, m1, v1 = ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    out2, m2, v2 = ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    terms = torch.empty((1, 5), dtype=torch.float64, device="cuda")
    ctx.step(th, out1, m1, v1, 1, lr=1e-2, terms=terms)
    t2, g = ctx.loss_grad(th)
    ctx.adam(th, out2, m2, v2, g, 1, lr=1e-2)
    torch.cuda.synchronize()
    assert torch.equal(out1, out2) and torch.equal(m1, m2) and torch.equal(v1, v2)
    assert torch.equal(terms, t2)
    rterms, _ = ops.loss_and_grad(spec, lv)
    assert_terms(terms[0].cpu().numpy(), rterms, 1e-5, op)


def test_run_argument_errors():
    need_gpu()
    from paper_2303_04679_amd import _lib as L
    spec = case("poisson", (16, 16), 2, seed=1)
    ctx = context_of(spec, "f64")
    a, b, m, v = ctx.new_pack(), ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    for args in ((a, a, m, v, 1, 3), (a, b, m, v, 1, 0), (a, b, m, v, 0, 2)):
        with pytest.raises(L.ModilError) as ei:
            ctx.run(*args)
        assert ei.value.status == L.ERR_INVALID_ARG


def test_deterministic():
    need_gpu()
    spec = case("ns3d", (16, 16, 16), 3, seed=9, with_forcing=True)
    ctx = context_of(spec, "f32")
    theta = pack_of(ctx, [_levels(spec, 10)])
    t1, g1 = ctx.loss_grad(theta)
    t2, g2 = ctx.loss_grad(theta)
    torch.cuda.synchronize()
    assert torch.equal(t1, t2) and torch.equal(g1, g2)


def test_batch_instances():
    """Independent instances with their own data and Reynolds number."""
    need_gpu()
    specs = []
    for b in range(3):
        s = case("cavity", (32, 32), 3, seed=20 + b)
        s.params["re"] = 100.0 + 300.0 * b
        specs.append(s)
    ctx = context_of(specs[0], "f64", batch=3, specs=specs)
    lvs = [_levels(s, 30 + b) for b, s in enumerate(specs)]
    theta = pack_of(ctx, lvs)
    terms, grad = ctx.loss_grad(theta)
    r = ctx.residual_metric(theta)
    torch.cuda.synchronize()
    for b, s in enumerate(specs):
        rt, rg = ops.loss_and_grad(s, lvs[b])
        assert_terms(terms[b].cpu().numpy(), rt, 1e-12, b)
        assert_levels(levels_of(ctx, grad, b), rg, 1e-12, b)
        assert abs(float(r[b]) - ops.residual_metric(s, lvs[b])) <= 1e-12 * float(r[b])


def test_nonfinite_is_reported():
    """A NaN measurement (forced from the host) raises MODIL_ERR_NONFINITE at check()."""
    need_gpu()
    from paper_2303_04679_amd import _lib as L
    spec = case("burgers", (16, 16), 2, seed=1)
    f, term, idx, vals, w = spec.meas[0]
    vals = vals.copy()
    vals[0] = float("nan")
    spec.meas = [(f, term, idx, vals, w)]
    ctx = context_of(spec, "f64")
    theta = pack_of(ctx, [_levels(spec, 2)])
    ctx.loss(theta)
    with pytest.raises(L.ModilError) as ei:
        ctx.check()
    assert ei.value.status == L.ERR_NONFINITE
    ctx.check()   # the flag is cleared


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("op,dims,L,batch", [("heat", (40, 72), 3, 1), ("cavity", (32, 48), 4, 1),
                                             ("burgers", (24, 40), 3, 1), ("poisson", (32, 48), 4, 1),
                                             ("poisson_node", (16, 24), 3, 1), ("cavity_node", (32, 48), 4, 1),
                                             ("cavity_node", (48, 64), 3, 12),
                                             ("heat", (64, 96), 3, 12), ("cavity", (48, 64), 3, 16),
                                             ("poisson", (24, 40), 2, 1), ("burgers", (16, 24), 1, 1),
                                             ("cavity_node", (16, 32), 2, 1), ("heat", (32, 48), 2, 1)])
def test_tiled_engine(op, dims, L, batch, dtype):
    """The 2-D tiled engine (16 x 4 tiles; 32 x 8 when the batch fills the
    chip), which forms the finest level theta_0 + T w_1 itself while staging,
    against the per-cell kernel for every instance and the oracle for the
    first and last; ragged tiles, node-based values, an x-only field, two
    levels (w_1 is theta_1) and one (no prolongation)."""
    need_gpu()
    print(f"\n[parity] tiled {op} {dims} L={L} batch={batch} {dtype}", flush=True)
    forcing = op not in ("poisson", "poisson_node")
    specs = [case(op, dims, L, seed=60 + b, with_forcing=forcing) for b in range(batch)]
    ctx = context_of(specs[0], dtype, batch=batch, specs=specs)
    lvs = [rounded(_levels(s, 70 + b), dtype) for b, s in enumerate(specs)]
    theta = pack_of(ctx, lvs)
    tt, gt = ctx.loss_grad(theta)
    lt = ctx.loss(theta)
    ctx.set_tile(False)
    tc, gc = ctx.loss_grad(theta)
    torch.cuda.synchronize()
    tol = TOL[dtype]
    for b in range(batch):
        ref = {t: float(tc[b, k]) for k, t in enumerate(TERMS)}
        assert_terms(tt[b].cpu().numpy(), ref, tol, ("per-cell", b))
        assert_terms(lt[b].cpu().numpy(), ref, tol, ("per-cell loss", b))
        assert_levels(levels_of(ctx, gt, b), levels_of(ctx, gc, b), tol, ("per-cell", b))
    for b in sorted({0, batch - 1}):
        rt, rg = ops.loss_and_grad(specs[b], lvs[b])
        assert_terms(tt[b].cpu().numpy(), rt, tol, ("oracle", b))
        assert_levels(levels_of(ctx, gt, b), rg, tol, ("oracle", b))


def test_theta_pingpong_required():
    need_gpu()
    from paper_2303_04679_amd import _lib as L
    spec = case("poisson", (16, 16), 2, seed=1)
    ctx = context_of(spec, "f64")
    a, m, v = ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    with pytest.raises(L.ModilError) as ei:
        ctx.step(a, a, m, v, 1)
    assert ei.value.status == L.ERR_INVALID_ARG


@pytest.mark.parametrize("op,dims,L", [("ns3d", (24, 36, 60), 3), ("ns3d_fixed", (16, 28, 24), 3),
                                       ("ns3d", (64, 16, 32), 4), ("ns3d", (8, 8, 8), 1)])
def test_fused_channel_kernel(op, dims, L):
    """The fused channel-flow pass (FP32; ragged xy tiles, several z-chunks)
    matches the oracle and the generic engine, for loss_grad and for the full
    step."""
    need_gpu()
    dtype = "f32"
    print(f"\n[parity] fused {op} {dims} L={L} {dtype}", flush=True)
    spec = case(op, dims, L, seed=13, with_forcing=True)
    lv = rounded(_levels(spec, 14), dtype)
    rterms, rgrad = ops.loss_and_grad(spec, lv)
    ctx = context_of(spec, dtype)
    assert ctx.fused_active()
    theta = pack_of(ctx, [lv])
    tf, gf = ctx.loss_grad(theta)
    ctx.set_fused(False)
    assert not ctx.fused_active()
    tg, gg = ctx.loss_grad(theta)
    torch.cuda.synchronize()
    tol = TOL[dtype]
    assert_terms(tf[0].cpu().numpy(), rterms, tol, "fused")
    assert_levels(levels_of(ctx, gf), rgrad, tol, "fused")
    assert_terms(tg[0].cpu().numpy(), rterms, tol, "generic")
    assert_levels(levels_of(ctx, gf), levels_of(ctx, gg), tol, "fused vs generic")
    # full step: fused Adam on every level against the generic step
    outs = []
    for fused in (True, False):
        ctx.set_fused(fused)
        o, m, v = ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
        ctx.step(theta, o, m, v, 1, lr=1e-2)
        ctx.step(o, theta.clone(), m, v, 2, lr=1e-2)
        outs.append((o, m, v))
    torch.cuda.synchronize()
    # in FP32 Adam's first steps are sign-like for near-zero gradients: compare m, v only
    for a, b in list(zip(outs[0], outs[1]))[1:]:
        assert_levels(levels_of(ctx, a), levels_of(ctx, b), tol, "step")
    # after one fused step from zero moments m = (1 - b1) g with g the oracle's gradient
    o, m, v = ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    ctx.set_fused(True)
    ctx.step(theta, o, m, v, 1, lr=1e-2)
    torch.cuda.synchronize()
    assert_levels(levels_of(ctx, m), [[0.1 * g for g in row] for row in rgrad], tol, "fused m", spec=spec)


def test_fused_channel_kernel_fp32_only():
    """FP64 channel flow runs on the generic engine (the fused kernel is FP32)."""
    need_gpu()
    spec = case("ns3d", (16, 16, 16), 2, seed=3)
    assert not context_of(spec, "f64").fused_active()
    assert context_of(spec, "f32").fused_active()


@pytest.mark.parametrize("batch", [4, 26, 52, 86, 130])
def test_fused_channel_zchunks(batch):
    """z-chunk lengths 2, 4, 8, 16 and 32: a batch of one-tile instances with
    40 planes (the longer chunks end ragged).  The chunk is the longest that
    gives every compute unit a block, so these batch sizes select the lengths.
    Every instance matches the generic engine; the first and last the oracle
    (FP32 inputs, promoted to FP64 for the oracle)."""
    need_gpu()
    dims = (40, 12, 20)
    print(f"\n[parity] fused z-chunks {dims} batch={batch}", flush=True)
    specs = [case("ns3d", dims, 3, seed=300 + b) for b in range(batch)]
    ctx = context_of(specs[0], "f32", batch=batch, specs=specs)
    assert ctx.fused_active()
    lvs = [rounded(_levels(s, 400 + b), "f32") for b, s in enumerate(specs)]
    theta = pack_of(ctx, lvs)
    tf, gf = ctx.loss_grad(theta)
    ctx.set_fused(False)
    tg, gg = ctx.loss_grad(theta)
    torch.cuda.synchronize()
    tol = TOL["f32"]
    for b in range(batch):
        assert_terms(tf[b].cpu().numpy(), {t: float(tg[b, k]) for k, t in enumerate(TERMS)},
                     tol, ("generic", b))
        assert_levels(levels_of(ctx, gf, b), levels_of(ctx, gg, b), tol, ("generic", b))
    for b in (0, batch - 1):
        rt, rg = ops.loss_and_grad(specs[b], lvs[b])
        assert_terms(tf[b].cpu().numpy(), rt, tol, ("oracle", b))
        assert_levels(levels_of(ctx, gf, b), rg, tol, ("oracle", b))


def test_fused_channel_batch():
    need_gpu()
    specs = [case("ns3d", (16, 24, 32), 3, seed=40 + b) for b in range(2)]
    ctx = context_of(specs[0], "f32", batch=2, specs=specs)
    assert ctx.fused_active()
    lvs = [rounded(_levels(s, 50 + b), "f32") for b, s in enumerate(specs)]
    theta = pack_of(ctx, lvs)
    terms, grad = ctx.loss_grad(theta)
    torch.cuda.synchronize()
    for b, s in enumerate(specs):
        rt, rg = ops.loss_and_grad(s, lvs[b])
        assert_terms(terms[b].cpu().numpy(), rt, TOL["f32"], b)
        assert_levels(levels_of(ctx, grad, b), rg, TOL["f32"], b)


@pytest.mark.parametrize("op,dims,L,dtype", [("cavity", (32, 48), 4, "f32"), ("heat", (32, 64), 4, "f64"),
                                             ("cavity_node", (32, 48), 4, "f64"),
                                             ("ns3d", (16, 16, 32), 3, "f32"),
                                             ("ns3d_node", (16, 16, 32), 3, "f32")])
@pytest.mark.parametrize("n", [1, 4, 5])
def test_run_equals_steps(op, dims, L, dtype, n):
    """modil_run of n iterations equals n modil_step calls bit for bit
    (packs, moments and the last loss terms)."""
    _run_equals_steps(op, dims, L, dtype, n)


@pytest.mark.parametrize("op,dims,L,dtype", [("ns3d", (32, 32, 64), 4, "f32"),
                                             ("cavity", (128, 128), 5, "f32"),
                                             ("cavity_node", (64, 64), 4, "f64"),
                                             ("heat", (256, 256), 6, "f64"),
                                             ("ns3d", (128, 128, 128), 6, "f32"),
                                             ("ns3d_node", (64, 64, 128), 6, "f32")])
def test_run_equals_steps_split_tail(op, dims, L, dtype):
    """Sizes whose Horner tail splits its largest level over several blocks per
    field, evenly or not (the restriction tail carries that split from one
    iteration to the next; the 128^3 channel flow is the benchmark workload):
    modil_run of 4 iterations equals 4 modil_step calls bit for bit."""
    _run_equals_steps(op, dims, L, dtype, 4)


def _run_equals_steps(op, dims, L, dtype, n):
    need_gpu()
    print(f"\n[parity] run == steps {op} {dims} L={L} {dtype} n={n}", flush=True)
    spec = case(op, dims, L, seed=21, with_forcing=op != "poisson")
    lv = rounded(_levels(spec, 22), dtype)
    ctx = context_of(spec, dtype)
    th0 = pack_of(ctx, [lv])
    a, b, m, v = th0.clone(), ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    t_run = torch.empty((1, 5), dtype=torch.float64, device="cuda")
    res = ctx.run(a, b, m, v, 3, n, lr=1e-3, terms=t_run)
    assert res is (b if n % 2 else a)
    a2, b2, m2, v2 = th0.clone(), ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    t_step = torch.empty((1, 5), dtype=torch.float64, device="cuda")
    for k in range(n):
        ctx.step(a2, b2, m2, v2, 3 + k, lr=1e-3, terms=t_step)
        a2, b2 = b2, a2
    torch.cuda.synchronize()
    assert torch.equal(res, a2) and torch.equal(m, m2) and torch.equal(v, v2)
    assert torch.equal(t_run, t_step)
