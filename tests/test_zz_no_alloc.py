"""The allocation-free prolongation (modil_prolong_noalloc) through the C ABI:
the same fine fields as modil_prolong with a context's workspace, bit for bit,
on two calls in a row (the second with a smaller problem, so the scratch holds
the first call's values), and the size limit."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import multigrid as mg
from oracle import operators as ops
from paper_2303_04679_amd import _lib as L
from paper_2303_04679_amd.modil import Context, ProblemSpec

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _noalloc(spec, theta, out):
    p = spec.to_c()
    stream = torch.cuda.current_stream()
    return L.lib().modil_prolong_noalloc(ctypes.byref(p), _ptr(theta), _ptr(out),
                                         ctypes.c_void_p(stream.cuda_stream))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_prolong_noalloc_equals_prolong(dtype):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cases = [ProblemSpec("ns3d", (32, 48, 64), (1.0, 1.0, 1.0), 4, dtype=dtype, max_meas=1, re=60.0),
             ProblemSpec("cavity", (32, 16), (1.0, 1.0), 3, dtype=dtype, batch=3, max_meas=1)]
    for spec in cases:   # the second problem is smaller than the first
        print(f"\n[noalloc] prolong {spec.op} {tuple(spec.dims)} L={spec.n_levels} {dtype} "
              f"batch={spec.batch}", flush=True)
        ctx = Context(spec)
        g = torch.Generator(device="cpu").manual_seed(7)
        theta = torch.rand(int(ctx.lay.total), generator=g, dtype=torch.float64).to(
            device="cuda", dtype=ctx.dtype) * 2 - 1
        ref = ctx.prolong(theta)
        torch.cuda.synchronize()
        out = torch.full_like(ref, float("nan"))
        assert _noalloc(spec, theta, out) == L.OK
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        # and the oracle's decomposition (FP64 values of the same inputs)
        for b in range(spec.batch):
            lv = [[v.double().cpu() for v in row] for row in ctx.level_views(theta, b)]
            for f, name in enumerate(spec.fields):
                axes = ops.field_axes(spec.op, name, len(spec.dims))
                want = mg.decompose_horner([row[f] for row in lv], axes, "cell").numpy()
                got = ctx.fine_views(out, b)[f].double().cpu().numpy()
                tol = 1e-14 if dtype == "f64" else 1e-6
                assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(want))
        ctx.close()


def test_prolong_noalloc_rejects_more_than_its_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    spec = ProblemSpec("ns3d", (256, 256, 256), (1.0, 1.0, 1.0), 7, dtype="f32", max_meas=1, re=60.0)
    theta = torch.zeros(16, device="cuda")
    with pytest.raises(L.ModilError) as ei:
        L.check(_noalloc(spec, theta, theta))
    assert ei.value.status == L.ERR_SHAPE
    assert "scratch" in str(ei.value)
