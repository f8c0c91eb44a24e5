"""Degenerate shapes on the HIP path, against the FP64 oracle: one level (the
decomposition is the identity), the coarsest level of exactly two cells per
axis (the cell-based prolongation then extrapolates at both ends of every
coarse row), the smallest grids the library accepts (four cells per axis,
smaller than one tile of every kernel), and problems without measurements
(the data term is exactly zero)."""
import numpy as np
import pytest
import torch

from oracle import adam as oadam
from oracle import operators as ops
from tests.gpu_helpers import TERMS, TOL, assert_levels, assert_terms, context_of, levels_of, need_gpu, pack_of, rounded
from tests.oracle_cases import case, random_levels

pytestmark = pytest.mark.gpu

SINGLE = [("poisson", (64,)), ("poisson", (16, 24)), ("poisson", (8, 4, 12)), ("burgers", (16, 24)),
          ("heat", (16, 8)), ("cavity", (16, 12)), ("ns3d", (8, 8, 8)), ("poisson_node", (12, 8)),
          ("cavity_node", (8, 12)), ("ns3d_node", (4, 8, 8))]
TWO_CELLS = [("poisson", (16,), 4), ("poisson", (8, 16), 3), ("burgers", (16, 16), 4), ("heat", (16, 32), 4),
             ("cavity", (16, 8), 3), ("ns3d", (8, 8, 16), 3), ("poisson_node", (16, 8), 3),
             ("cavity_node", (8, 16), 3)]
SMALLEST = [("poisson", (4,), 2), ("poisson", (4, 4, 4), 2), ("burgers", (4, 4), 2), ("heat", (4, 4), 2),
            ("cavity", (4, 4), 2), ("ns3d", (4, 4, 4), 2), ("ns3d", (4, 4, 4), 1), ("ns3d", (4, 8, 12), 2),
            ("cavity_node", (4, 4), 2)]


def _levels(spec, seed):
    if spec.op == "burgers":
        return random_levels(spec, seed, lo=0.05, hi=0.6)
    return random_levels(spec, seed)


def _loss_grad(op, dims, L, dtype, spec=None):
    spec = spec or case(op, dims, L, seed=17, with_forcing=op != "poisson")
    lv = rounded(_levels(spec, 18), dtype)
    ref_terms, ref_grad = ops.loss_and_grad(spec, lv)
    ctx = context_of(spec, dtype)
    terms, grad = ctx.loss_grad(pack_of(ctx, [lv]))
    torch.cuda.synchronize()
    got = terms[0].cpu().numpy()
    assert_terms(got, ref_terms, TOL[dtype], (op, dims, L))
    assert_levels(levels_of(ctx, grad), ref_grad, TOL[dtype], (op, dims, L))
    return got, ctx


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("op,dims", SINGLE)
def test_single_level(op, dims, dtype):
    need_gpu()
    print(f"\n[degenerate] one level {op} {dims} {dtype}", flush=True)
    _loss_grad(op, dims, 1, dtype)


@pytest.mark.parametrize("op,dims", SINGLE)
def test_single_level_steps_f64(op, dims):
    """Two FP64 iterations on one level follow the oracle's gradient and Adam."""
    need_gpu()
    print(f"\n[degenerate] one level, two steps {op} {dims}", flush=True)
    spec = case(op, dims, 1, seed=19, with_forcing=op != "poisson")
    lv = _levels(spec, 20)
    ctx = context_of(spec, "f64")
    a, b, m, v = pack_of(ctx, [lv]), ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    ref = [(x.copy(), np.zeros_like(x), np.zeros_like(x)) for x in lv[0]]
    terms = torch.empty((1, 5), dtype=torch.float64, device="cuda")
    for t in (1, 2):
        ctx.step(a, b, m, v, t, lr=1e-2, terms=terms)
        torch.cuda.synchronize()
        rterms, rgrad = ops.loss_and_grad(spec, [[s[0] for s in ref]])
        assert_terms(terms[0].cpu().numpy(), rterms, 1e-12, (op, t))
        ref = [oadam.adam_step(s[0], s[1], s[2], g, 1e-2, 0.9, 0.999, 1e-8, t) for s, g in zip(ref, rgrad[0])]
        a, b = b, a
    for name, pk, k in (("theta", a, 0), ("m", m, 1), ("v", v, 2)):
        assert_levels(levels_of(ctx, pk), [[s[k] for s in ref]], 1e-12, (op, name))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("op,dims,L", TWO_CELLS)
def test_coarsest_level_of_two_cells(op, dims, L, dtype):
    need_gpu()
    print(f"\n[degenerate] two coarsest cells {op} {dims} L={L} {dtype}", flush=True)
    _loss_grad(op, dims, L, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("op,dims,L", SMALLEST)
def test_smallest_grids(op, dims, L, dtype):
    need_gpu()
    print(f"\n[degenerate] smallest grid {op} {dims} L={L} {dtype}", flush=True)
    _, ctx = _loss_grad(op, dims, L, dtype)
    if op == "ns3d" and dtype == "f32":
        assert ctx.fused_active()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("op,dims,L", [("cavity", (32, 16), 3), ("ns3d", (16, 8, 24), 3),
                                       ("burgers", (32, 32), 3), ("cavity_node", (16, 16), 3)])
def test_no_measurements(op, dims, L, dtype):
    need_gpu()
    print(f"\n[degenerate] no measurements {op} {dims} L={L} {dtype}", flush=True)
    spec = case(op, dims, L, seed=21, with_forcing=True)
    spec.meas = []
    got, ctx = _loss_grad(op, dims, L, dtype, spec=spec)
    assert got[TERMS.index("data")] == 0.0
    if op == "ns3d" and dtype == "f32":
        assert ctx.fused_active()
