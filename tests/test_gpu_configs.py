"""Parity at the full sizes of the benchmark workloads (and of one GPU's share
of the 128^3 channel flow), through the same contexts bench.py times (fused
channel-flow path for the 3-D problems)."""
import numpy as np
import pytest
import torch

from oracle import operators as ops
from paper_2303_04679_amd import configs, synth
from tests.gpu_helpers import TOL, assert_levels, assert_terms, levels_of, need_gpu, pack_of, rounded
from tests.workload_oracle import oracle_spec

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["burgers64", "heat256", "heat256_f32", "ns3d64", "ns3d128", "ns3d256",
                                  "ns3d128_shard8", "cavity128", "channel_node129"])
def test_workload_loss_and_gradient(name):
    need_gpu()
    print(f"\n[parity] workload {name}", flush=True)
    wl = configs.WORKLOADS[name]()
    ctx, theta0 = configs.build(wl)
    spec = oracle_spec(wl)
    shapes = ops.level_shapes(spec.op, spec.dims, spec.n_levels, spec.centering)
    lv = synth.uniform_levels(shapes, 90, -0.5, 0.5)
    # start from the workload's own initial state plus a random perturbation
    base = [[v.detach().cpu().double().numpy() for v in row] for row in ctx.level_views(theta0)]
    lv = rounded([[b + x for b, x in zip(br, xr)] for br, xr in zip(base, lv)], wl.spec.dtype)
    theta = pack_of(ctx, [lv])
    terms, grad = ctx.loss_grad(theta)
    torch.cuda.synchronize()
    rterms, rgrad = ops.loss_and_grad(spec, lv)
    tol = TOL[wl.spec.dtype]
    assert_terms(terms[0].cpu().numpy(), rterms, tol, name)
    assert_levels(levels_of(ctx, grad), rgrad, tol, name,
                  spec=spec if wl.spec.dtype == "f32" else None)
