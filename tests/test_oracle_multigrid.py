"""Pins of the oracle's multigrid decomposition (paper Section 2.2)."""
import os

import numpy as np
import pytest
import torch

from oracle import multigrid as mg

GOLD = os.path.join(os.path.dirname(__file__), "golden", "interp_matrices.txt")


def _read_golden():
    mats, name, scale, rows = {}, None, None, []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        if parts[0][0].isalpha():
            if name:
                mats[name] = scale * np.array(rows, dtype=float)
            name, scale, rows = parts[0], float(parts[1]), []
        else:
            rows.append([int(p) for p in parts])
    mats[name] = scale * np.array(rows, dtype=float)
    return mats


def test_printed_matrices():
    """T matrices equal the paper's printed ones (node 9x5, 5x3; cell 8x4, 4x2)."""
    g = _read_golden()
    np.testing.assert_array_equal(mg.node_T_matrix(4), g["node_T1"])
    np.testing.assert_array_equal(mg.node_T_matrix(2), g["node_T2"])
    np.testing.assert_array_equal(mg.cell_T_matrix(4), g["cell_T1"])
    np.testing.assert_array_equal(mg.cell_T_matrix(2), g["cell_T2"])


@pytest.mark.parametrize("centering,n", [("cell", 2), ("cell", 3), ("cell", 4), ("cell", 16),
                                         ("node", 2), ("node", 4), ("node", 8)])
def test_slicing_forms_match_dense(centering, n):
    """The slicing prolongation and restriction are T and T^T column by column."""
    T = mg.cell_T_matrix(n) if centering == "cell" else mg.node_T_matrix(n)
    m = T.shape[1]
    eye = torch.eye(m, dtype=torch.float64)
    P = mg.prolong_axis(eye, 0, centering).numpy()
    np.testing.assert_array_equal(P, T)
    eyef = torch.eye(T.shape[0], dtype=torch.float64)
    R = mg.restrict_axis(eyef, 0, centering).numpy()
    np.testing.assert_array_equal(R, T.T)


def test_rows_sum_to_one():
    """Linear interpolation reproduces constants: every row of T sums to 1."""
    for n in (2, 3, 5, 8):
        np.testing.assert_allclose(mg.cell_T_matrix(n).sum(1), 1.0, rtol=0, atol=0)
        np.testing.assert_allclose(mg.node_T_matrix(n).sum(1), 1.0, rtol=0, atol=0)


def test_cell_T_exact_on_linear():
    """Cell-based T (with its extrapolated end rows) is exact for linear functions."""
    n = 6
    xc = (np.arange(n) + 0.5) / n
    xf = (np.arange(2 * n) + 0.5) / (2 * n)
    f = lambda x: 3.0 * x - 1.25
    np.testing.assert_allclose(mg.cell_T_matrix(n) @ f(xc), f(xf), rtol=0, atol=1e-14)


@pytest.mark.parametrize("centering", ["cell", "node"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_horner_equals_direct_and_dense(centering, ndim):
    """Horner form = direct sum = Kronecker-product matrix (Section 2.2)."""
    n, L = 8, 3
    rng = np.random.default_rng(ndim)
    sizes = mg.level_sizes(n, L)
    ext = (lambda s: s) if centering == "cell" else (lambda s: s + 1)
    levels = [torch.tensor(rng.standard_normal((ext(s),) * ndim)) for s in sizes]
    axes = tuple(range(ndim))
    h = mg.decompose_horner(levels, axes, centering).numpy()
    d = mg.decompose_direct(levels, axes, centering).numpy()
    np.testing.assert_allclose(h, d, rtol=0, atol=1e-13)
    M = mg.dense_decomposition_matrix(n, L, ndim, centering)
    flat = np.concatenate([lv.numpy().ravel() for lv in levels])
    np.testing.assert_allclose(M @ flat, h.ravel(), rtol=0, atol=1e-13)


@pytest.mark.parametrize("centering", ["cell", "node"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_adjoint_identity(centering, ndim):
    """<M u, v> = sum_l <u_l, (M^T v)_l>, and M^T equals the dense transpose."""
    n, L = 16 if ndim < 3 else 8, 4 if ndim < 3 else 3
    rng = np.random.default_rng(10 + ndim)
    sizes = mg.level_sizes(n, L)
    ext = (lambda s: s) if centering == "cell" else (lambda s: s + 1)
    axes = tuple(range(ndim))
    levels = [torch.tensor(rng.standard_normal((ext(s),) * ndim)) for s in sizes]
    v = torch.tensor(rng.standard_normal((ext(n),) * ndim))
    lhs = float((mg.decompose_horner(levels, axes, centering) * v).sum())
    adj = mg.decompose_transpose(v, L, axes, centering)
    rhs = sum(float((a * b).sum()) for a, b in zip(levels, adj))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    M = mg.dense_decomposition_matrix(n, L, ndim, centering)
    flat = np.concatenate([a.numpy().ravel() for a in adj])
    np.testing.assert_allclose(M.T @ v.numpy().ravel(), flat, rtol=0, atol=1e-12)


def test_end_column_sums():
    """Columns 0 and n-1 of the cell-based T sum to 9/4, columns 1 and n-2 to 7/4."""
    T = mg.cell_T_matrix(8)
    s = T.sum(0)
    assert s[0] == s[-1] == 2.25
    assert s[1] == s[-2] == 1.75
    assert np.all(s[2:-2] == 2.0)


def test_level_sizes():
    assert mg.level_sizes(64, 5) == [64, 32, 16, 8, 4]
    with pytest.raises(ValueError):
        mg.level_sizes(24, 5)
