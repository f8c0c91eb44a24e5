"""The data-only loss (every weight but the data weight at zero) on the HIP
path.  With the operator switched off, the loss gradient is M_L^T applied to
the point misfits 2 w (u - y) alone, so these cases isolate the
prolongation, the measurement gather and scatter, and the restriction from
the finite-difference residuals.

Two checks: the terms and gradient against the FP64 oracle, and, without the
oracle, the gradient against the library's own restriction of a fine misfit
vector assembled on the host from the library's prolongation.
"""
import numpy as np
import pytest
import torch

from oracle import operators as ops
from tests.gpu_helpers import TOL, assert_levels, assert_terms, context_of, levels_of, need_gpu, pack_of, rel, rounded
from tests.oracle_cases import case, random_levels

pytestmark = pytest.mark.gpu

CASES = [("cavity", (32, 48), 4), ("ns3d", (16, 16, 24), 3), ("heat", (40, 72), 3),
         ("burgers", (64, 64), 5), ("cavity_node", (24, 16), 3), ("ns3d_node", (8, 12, 20), 2)]


def _data_only(op, dims, L):
    spec = case(op, dims, L, seed=9)
    spec.weights = {t: 0.0 for t in spec.weights}
    spec.weights["data"] = 1.0
    spec.meas = [m for m in spec.meas if m[1] == "data"]
    return spec


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("op,dims,L", CASES)
def test_data_only_matches_oracle(op, dims, L, dtype):
    need_gpu()
    print(f"\n[null operator] {op} {dims} L={L} {dtype}", flush=True)
    spec = _data_only(op, dims, L)
    lv = rounded(random_levels(spec, 10), dtype)
    ref_terms, ref_grad = ops.loss_and_grad(spec, lv)
    assert ref_terms["data"] > 0.0
    ctx = context_of(spec, dtype)
    theta = pack_of(ctx, [lv])
    terms, grad = ctx.loss_grad(theta)
    torch.cuda.synchronize()
    got = terms[0].cpu().numpy()
    assert_terms(got, ref_terms, TOL[dtype], op)
    assert got[0] == 0.0
    assert_levels(levels_of(ctx, grad), ref_grad, TOL[dtype], op)


@pytest.mark.parametrize("op,dims,L", CASES)
def test_data_only_gradient_is_restricted_misfit(op, dims, L):
    """grad = M^T g with g = 2 w (u - y) at the measured points, u = M theta,
    both M and M^T taken from the library; FP64."""
    need_gpu()
    print(f"\n[null operator] restricted misfit {op} {dims} L={L}", flush=True)
    spec = _data_only(op, dims, L)
    lv = random_levels(spec, 11)
    ctx = context_of(spec, "f64")
    theta = pack_of(ctx, [lv])
    fine = ctx.prolong(theta)
    torch.cuda.synchronize()
    u = [v.cpu().numpy().reshape(-1) for v in ctx.fine_views(fine)]
    mis = [np.zeros_like(x) for x in u]
    for fi, _, idx, vals, wt in spec.meas:
        np.add.at(mis[fi], np.asarray(idx), 2.0 * wt * (u[fi][np.asarray(idx)] - vals))
    g = torch.zeros_like(fine)
    for v, m in zip(ctx.fine_views(g), mis):
        v.copy_(torch.tensor(m.reshape(v.shape), dtype=torch.float64))
    want = levels_of(ctx, ctx.restrict_adjoint(g))
    _, grad = ctx.loss_grad(theta)
    torch.cuda.synchronize()
    got = levels_of(ctx, grad)
    for li in range(L):
        for f in range(len(spec.fields)):
            assert rel(got[li][f], want[li][f]) <= 1e-13, (li, f)
