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
    # the timed path: Adam fused into the finest and the restriction kernels;
    # two plain steps from zero moments, then the same two iterations in one
    # modil_run call (the second starting from the Horner tail the first
    # one's restriction tail carried)
    o1, o2 = ctx.new_pack(), ctx.new_pack()
    m, v = ctx.new_pack(), ctx.new_pack()
    t1 = torch.empty((1, 5), dtype=torch.float64, device="cuda")
    ctx.step(theta, o1, m, v, 1, lr=wl.lr, terms=t1)
    m1 = m.clone()
    ctx.step(o1, o2, m, v, 2, lr=wl.lr)
    ra, rb = theta.clone(), ctx.new_pack()
    rm, rv = ctx.new_pack(), ctx.new_pack()
    out = ctx.run(ra, rb, rm, rv, 1, 2, lr=wl.lr)
    torch.cuda.synchronize()
    assert torch.equal(out, o2) and torch.equal(rm, m) and torch.equal(rv, v), (name, "run == steps")
    rterms, rgrad = ops.loss_and_grad(spec, lv)
    tol = TOL[wl.spec.dtype]
    fspec = spec if wl.spec.dtype == "f32" else None
    assert_terms(terms[0].cpu().numpy(), rterms, tol, name)
    assert_levels(levels_of(ctx, grad), rgrad, tol, name, spec=fspec)
    # the first step's loss terms are those at theta; its first moment is
    # (1 - b1) times the oracle's gradient on every level
    assert_terms(t1[0].cpu().numpy(), rterms, tol, (name, "step"))
    assert_levels(levels_of(ctx, m1), [[0.1 * g for g in row] for row in rgrad], tol, (name, "step m"),
                  spec=fspec)
