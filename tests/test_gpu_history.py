"""Two integration checks of the optimizer loop.

Loss history: twenty modil_step iterations in FP64 follow the oracle's loss,
gradient and Adam step by step; every iteration's loss terms agree to 1e-12
relative, the FP64 parity bar (measured: at most about 1.4e-15 over the
twenty iterations on these grids).

Checkpoint and resume: theta, m and v written to disk after some modil_run
iterations and read back into fresh device buffers continue the run bit for
bit, so the pack state is the optimizer's whole state (the carried Horner
tail is rebuilt at the start of every call)."""
import numpy as np
import pytest
import torch

from oracle import adam as oadam
from oracle import operators as ops
from tests.gpu_helpers import TERMS, assert_terms, context_of, need_gpu, pack_of, rounded
from tests.oracle_cases import case
from tests.test_gpu_parity import _levels

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("op,dims,L", [("burgers", (32, 32), 4), ("heat", (32, 32), 4),
                                       ("cavity", (32, 32), 4), ("ns3d", (8, 8, 16), 3),
                                       ("poisson_node", (32, 32), 4)])
def test_loss_history_follows_oracle(op, dims, L):
    need_gpu()
    print(f"\n[history] {op} {dims} L={L}", flush=True)
    spec = case(op, dims, L, seed=5)
    lv = _levels(spec, 6)
    ctx = context_of(spec, "f64")
    a, b = pack_of(ctx, [lv]), ctx.new_pack()
    m, v = ctx.new_pack(), ctx.new_pack()
    ref = [[(x.copy(), np.zeros_like(x), np.zeros_like(x)) for x in row] for row in lv]
    terms = torch.empty((1, 5), dtype=torch.float64, device="cuda")
    worst = 0.0
    for t in range(1, 21):
        ctx.step(a, b, m, v, t, lr=1e-2, terms=terms)
        torch.cuda.synchronize()
        rterms, rgrad = ops.loss_and_grad(spec, [[s[0] for s in row] for row in ref])
        got = terms[0].cpu().numpy()
        for i, k in enumerate(TERMS):
            if rterms[k]:
                worst = max(worst, abs(got[i] - rterms[k]) / abs(rterms[k]))
        assert_terms(got, rterms, 1e-12, (op, t))
        ref = [[oadam.adam_step(s[0], s[1], s[2], g, 1e-2, 0.9, 0.999, 1e-8, t)
                for s, g in zip(row, grow)] for row, grow in zip(ref, rgrad)]
        a, b = b, a
    print(f"[history] worst relative term difference over 20 iterations {worst:.2e}", flush=True)


@pytest.mark.parametrize("op,dims,L,dtype", [("cavity", (32, 48), 4, "f32"),
                                             ("ns3d", (16, 16, 32), 3, "f32"),
                                             ("heat", (32, 64), 4, "f64")])
def test_checkpoint_resume_bitwise(op, dims, L, dtype, tmp_path):
    need_gpu()
    spec = case(op, dims, L, seed=21, with_forcing=op != "poisson")
    lv = rounded(_levels(spec, 22), dtype)
    ctx = context_of(spec, dtype)
    th0 = pack_of(ctx, [lv])
    # uninterrupted: 10 iterations from step 1
    a, b, m, v = th0.clone(), ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    full = ctx.run(a, b, m, v, 1, 10, lr=1e-3)
    # 4 iterations, checkpoint to disk, fresh buffers, 6 more from step 5
    a2, b2, m2, v2 = th0.clone(), ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    mid = ctx.run(a2, b2, m2, v2, 1, 4, lr=1e-3)
    torch.cuda.synchronize()
    path = tmp_path / "state.npz"
    np.savez(path, theta=mid.cpu().numpy(), m=m2.cpu().numpy(), v=v2.cpu().numpy(), step=5)
    del a2, b2, m2, v2, mid
    st = np.load(path)
    dev = lambda x: torch.from_numpy(x).to("cuda")
    a3, b3, m3, v3 = dev(st["theta"]), ctx.new_pack(), dev(st["m"]), dev(st["v"])
    res = ctx.run(a3, b3, m3, v3, int(st["step"]), 6, lr=1e-3)
    torch.cuda.synchronize()
    assert torch.equal(res, full) and torch.equal(m3, m) and torch.equal(v3, v)
