"""Engine variants and host checks of the generic path against each other and
the oracle: the two-pass 3-D adjoint against the per-cell kernel, the
node-based Horner step of 3-D fields, the residual metric of every operator,
and the rejection of measurements on boundary nodes."""
import numpy as np
import pytest
import torch

from oracle import multigrid as mg
from oracle import operators as ops
from paper_2303_04679_amd import _lib as L
from tests.gpu_helpers import assert_levels, assert_terms, context_of, levels_of, need_gpu, pack_of, rel
from tests.oracle_cases import case, random_levels

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("op,dims,lv", [("ns3d_node", (8, 12, 20), 2), ("ns3d_fixed_node", (8, 16, 24), 3),
                                        ("ns3d", (8, 16, 24), 3), ("ns3d_fixed", (16, 8, 16), 3),
                                        ("poisson", (16, 8, 24), 3), ("poisson_node", (8, 16, 8), 2)])
def test_two_pass_adjoint_equals_per_cell_kernel(op, dims, lv):
    """FP64: the gradient from per-cell star sensitivities and their gather
    equals the per-cell kernel's (which forms every neighbour's residuals
    again) to rounding, and both match the oracle."""
    need_gpu()
    print(f"\n[engine] two-pass vs per-cell {op} {dims} L={lv}", flush=True)
    spec = case(op, dims, lv, seed=13, with_forcing=op != "poisson" and op != "poisson_node")
    levels = random_levels(spec, 14)
    ctx = context_of(spec, "f64")
    theta = pack_of(ctx, [levels])
    t2, g2 = ctx.loss_grad(theta)
    ctx.set_two_pass(False)
    t1, g1 = ctx.loss_grad(theta)
    torch.cuda.synchronize()
    a, b = levels_of(ctx, g1), levels_of(ctx, g2)
    for li, (ra, rb) in enumerate(zip(a, b)):
        for fi, (x, y) in enumerate(zip(ra, rb)):
            assert rel(y, x) <= 1e-14, (op, li, fi, rel(y, x))
    assert torch.allclose(t1, t2, rtol=1e-14, atol=0)
    rterms, rgrad = ops.loss_and_grad(spec, levels)
    assert_terms(t2[0].cpu().numpy(), rterms, 1e-12, op)
    assert_levels(b, rgrad, 1e-12, op)


@pytest.mark.parametrize("op,dims,lv", [("poisson_node", (16, 32, 64), 3), ("poisson_node", (16, 16, 32), 4),
                                        ("ns3d_node", (8, 16, 32), 3), ("ns3d_node", (16, 8, 8), 2)])
def test_node_prolongation_of_3d_fields(op, dims, lv):
    """The node-based Horner step of fields spanning three axes (uneven node
    counts, e.g. 17 x 33 x 65) equals the oracle's decomposition."""
    need_gpu()
    print(f"\n[engine] node prolongation {op} {dims} L={lv}", flush=True)
    spec = case(op, dims, lv, seed=3)
    levels = random_levels(spec, 4)
    ctx = context_of(spec, "f64")
    fine = ctx.prolong(pack_of(ctx, [levels]))
    torch.cuda.synchronize()
    for f, name in enumerate(spec.fields):
        axes = ops.field_axes(spec.op, name, spec.ndim)
        ref = mg.decompose_horner([torch.tensor(r[f]) for r in levels], axes, "node").numpy()
        got = ctx.fine_views(fine)[f].cpu().numpy()
        assert got.shape == ref.shape
        assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref)), (op, f)


@pytest.mark.parametrize("op,dims,lv", [("burgers", (32, 48), 3), ("heat", (40, 24), 3),
                                        ("poisson", (16, 24), 3), ("poisson_node", (16, 8, 16), 2),
                                        ("cavity", (32, 32), 3), ("cavity_node", (24, 16), 3),
                                        ("ns3d", (8, 16, 16), 2), ("ns3d_node", (8, 12, 20), 2)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_residual_metric_every_operator(op, dims, lv, dtype):
    """r = RMS of the integrated residual over the points that carry the PDE
    equations (every cell, the interior nodes, or the inner space-time points)."""
    need_gpu()
    spec = case(op, dims, lv, seed=5, with_forcing=op not in ("poisson", "poisson_node"))
    levels = random_levels(spec, 6, lo=0.05, hi=0.6) if op == "burgers" else random_levels(spec, 6)
    if dtype == "f32":
        levels = [[np.asarray(x, dtype=np.float32).astype(np.float64) for x in row] for row in levels]
    ctx = context_of(spec, dtype)
    r = ctx.residual_metric(pack_of(ctx, [levels]))
    torch.cuda.synchronize()
    ref = ops.residual_metric(spec, levels)
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert abs(float(r[0]) - ref) <= tol * ref, (op, float(r[0]), ref)


@pytest.mark.parametrize("op,dims", [("poisson_node", (16, 16)), ("cavity_node", (16, 16)),
                                     ("ns3d_node", (8, 8, 16))])
def test_measurement_on_a_boundary_node_is_rejected(op, dims):
    """Boundary nodes hold imposed values: a measurement there is an error,
    one on an interior node is accepted."""
    need_gpu()
    from paper_2303_04679_amd.modil import Context
    from tests.gpu_helpers import problem_of
    spec = case(op, dims, 2, seed=1)
    spec.meas = []
    prob = problem_of(spec, "f64")
    prob.max_meas = 8
    ctx = Context(prob)
    shape = tuple(d + 1 for d in dims)
    inner = np.ravel_multi_index(tuple(1 for _ in dims), shape)
    ctx.set_measurements(0, np.array([inner], dtype=np.int32), np.array([0.5]), 1.0)
    for corner in (0, int(np.prod(shape)) - 1, np.ravel_multi_index((1,) * (len(dims) - 1) + (0,), shape),
                   np.ravel_multi_index((0,) + (1,) * (len(dims) - 1), shape)):
        with pytest.raises(L.ModilError) as ei:
            ctx.set_measurements(0, np.array([corner], dtype=np.int32), np.array([0.5]), 1.0)
        assert ei.value.status == L.ERR_SHAPE
