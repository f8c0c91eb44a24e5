"""Host-side checks of libmodil: it loads, exports what the header declares,
validates problems and computes pack layouts (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import operators as ops
from paper_2303_04679_amd import _lib as L
from paper_2303_04679_amd.modil import ProblemSpec, field_shape, layout

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "modil.h")


def test_library_exports_every_declared_function():
    text = open(HEADER).read()
    names = set(re.findall(r"\b(modil_[a-z_]+)\s*\(", text))
    lib = L.lib()
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    assert len(names) >= 20
    assert lib.modil_abi_version() == 1


def test_status_strings():
    lib = L.lib()
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert lib.modil_status_str(s)


@pytest.mark.parametrize("op,dims,L_,fields", [
    ("poisson", (16, 16), 3, None), ("burgers", (64, 64), 5, None), ("heat", (256, 256), 6, None),
    ("ns3d", (16, 16, 16), 3, None), ("cavity", (128, 128), 5, None)])
def test_layout_matches_level_shapes(op, dims, L_, fields):
    spec = ProblemSpec(op, dims, (1.0,) * len(dims), L_, batch=3)
    lay = layout(spec)
    shapes = ops.level_shapes(op, dims, L_)
    total = 0
    for lvl in range(L_):
        assert lay.level_offset[lvl] == total
        per_inst = 0
        for f, shp in enumerate(shapes[lvl]):
            assert field_shape(spec, lay, lvl, f) == tuple(shp)
            assert lay.field_offset[lvl][f] == per_inst
            per_inst += int(np.prod(shp))
        assert lay.level_stride[lvl] == per_inst
        total += 3 * per_inst
    assert lay.total == total
    assert lay.fine_cells == int(np.prod(dims))
    assert lay.workspace_bytes > 0


def test_config_sizes():
    """Parameter counts of the five workloads (levels x fields)."""
    cases = {("burgers", (64, 64), 5): 5456, ("heat", (256, 256), 6): 87360 + 504,
             ("ns3d", (64,) * 3, 5): 5 * 299584, ("ns3d", (128,) * 3, 6): 5 * 2396736,
             ("cavity", (128, 128), 5): 3 * 21824}
    for (op, dims, nl), want in cases.items():
        assert layout(ProblemSpec(op, dims, (1.0,) * len(dims), nl)).total == want


@pytest.mark.parametrize("kw,status", [
    (dict(op="ns3d", dims=(16, 16), lengths=(1, 1), n_levels=2), L.ERR_SHAPE),
    (dict(op="poisson", dims=(24, 24), lengths=(1, 1), n_levels=5), L.ERR_SHAPE),
    (dict(op="poisson", dims=(16,), lengths=(1,), n_levels=5), L.ERR_SHAPE),
    (dict(op="poisson", dims=(16,), lengths=(-1,), n_levels=2), L.ERR_INVALID_ARG),
    (dict(op="cavity", dims=(16, 16), lengths=(1, 1), n_levels=2, batch=0), L.ERR_INVALID_ARG),
    (dict(op="cavity", dims=(16, 16), lengths=(1, 1), n_levels=2, re=0.0), L.ERR_INVALID_ARG),
    (dict(op="cavity", dims=(16, 16), lengths=(1, 1), n_levels=2, chi_fixed=True), L.ERR_INVALID_ARG),
])
def test_validation_errors(kw, status):
    with pytest.raises(L.ModilError) as ei:
        layout(ProblemSpec(**kw))
    assert ei.value.status == status
    assert L.lib().modil_last_error(None)


@pytest.mark.parametrize("op,dims,lengths", [("burgers", (16, 16), (1.0, 2.0)),
                                             ("heat", (16, 16), (0.02, 1.0))])
def test_node_centering_not_for_burgers_and_heat(op, dims, lengths):
    p = ProblemSpec(op, dims, lengths, 2).to_c()
    p.centering = L.NODE
    out = L.PackLayout()
    assert L.lib().modil_layout(ctypes.byref(p), ctypes.byref(out)) == L.ERR_DTYPE


def test_node_cavity_layout():
    """Node-based cavity: three fields of (dims >> l) + 1 values per axis."""
    lay = layout(ProblemSpec("cavity", (64, 64), (1.0, 1.0), 5, centering="node"))
    for l, n in enumerate((65, 33, 17, 9, 5)):
        assert [tuple(lay.field_dims[l][f])[1:] for f in range(3)] == [(n, n)] * 3
    assert lay.fine_cells == 65 * 65
    assert lay.total == 3 * sum(n * n for n in (65, 33, 17, 9, 5))


def test_node_channel_layout():
    """Node-based channel flow: five fields of (dims >> l) + 1 values per axis."""
    lay = layout(ProblemSpec("ns3d", (64, 64, 128), (1.0, 1.0, 2.0), 3, re=200.0, centering="node"))
    for l, (nz, nx) in enumerate(((65, 129), (33, 65), (17, 33))):
        assert [tuple(lay.field_dims[l][f]) for f in range(5)] == [(nz, nz, nx)] * 5
    assert lay.fine_cells == 65 * 65 * 129
    assert lay.total == 5 * sum(a * a * b for a, b in ((65, 129), (33, 65), (17, 33)))


def test_node_layout():
    """Node-based Poisson: (dims >> l) + 1 values per axis on level l."""
    lay = layout(ProblemSpec("poisson", (32, 16), (1.0, 1.0), 3, centering="node"))
    dims = [tuple(lay.field_dims[l][0])[1:] for l in range(3)]
    assert dims == [(33, 17), (17, 9), (9, 5)]
    assert lay.fine_cells == 33 * 17
    assert lay.total == 33 * 17 + 17 * 9 + 9 * 5


def test_workspace_holds_two_pass_scratch_only_where_it_runs():
    """The two-pass 3-D adjoint's face sensitivities (6 x 4 fields x cells)
    are reserved for node-based and FP64 channel flow, not for FP32
    cell-based channel flow, which runs the fused kernel (or the per-cell
    kernel)."""
    n = 128
    cells = n ** 3
    f32 = layout(ProblemSpec("ns3d", (n,) * 3, (1.0,) * 3, 6, dtype="f32")).workspace_bytes
    f64 = layout(ProblemSpec("ns3d", (n,) * 3, (1.0,) * 3, 6, dtype="f64")).workspace_bytes
    # FP32: the gradient pack and the Horner levels dominate, no 24 values per cell
    assert f32 < 12 * cells * 4
    assert f64 > 6 * 4 * cells * 8
    node = layout(ProblemSpec("ns3d", (32, 32, 64), (1.0, 1.0, 2.0), 3, dtype="f32",
                              centering="node")).workspace_bytes
    assert node > 6 * 4 * 33 * 33 * 65 * 4
    p3 = layout(ProblemSpec("poisson", (32, 32, 32), (1.0,) * 3, 3, dtype="f32")).workspace_bytes
    assert p3 > 6 * 32 ** 3 * 4
