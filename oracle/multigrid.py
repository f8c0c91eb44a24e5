"""Multigrid decomposition of a grid field (paper Section 2.2).

A field u on the finest grid (N_1 = N cells per axis) is represented by a
hierarchy of fields u_1..u_L on grids N_i = N / 2^(i-1), and

    u = M_L(u_1, ..., u_L) = u_1 + T_1 u_2 + ... + T_1 T_2 ... T_{L-1} u_L,

evaluated in Horner form u_1 + T_1(u_2 + T_2(u_3 + ...)).  T_i is linear
interpolation from grid N_{i+1} to grid N_i.  In d dimensions T is the tensor
product of the one-dimensional operator along every axis the field spans.

Two one-dimensional operators are given in the paper (Section 2.2, the
printed 9x5 / 5x3 node-based and 8x4 / 4x2 cell-based matrices):

  cell-based, n coarse cells -> 2n fine cells:
      interior fine cells are 3/4 of the parent cell plus 1/4 of the nearer
      neighbouring coarse cell; the two end fine cells use linear
      extrapolation, 5/4 of the end coarse cell minus 1/4 of its neighbour.
  node-based, n+1 coarse nodes -> 2n+1 fine nodes:
      even fine nodes copy the coincident coarse node, odd fine nodes are the
      mean of the two adjacent coarse nodes.

The transpose M_L^T maps a fine-grid field (for instance dL/du) to one field
per level: (M_L^T g)_l = T_{l-1}^T ... T_1^T g.  It is the exact transpose,
not an averaging restriction.
"""
import numpy as np
import torch

DT = torch.float64


def level_sizes(n, n_levels):
    """Cells per axis on each level, N_i = N / 2^(i-1) (Section 2.2)."""
    out = []
    for i in range(n_levels):
        if n % (2 ** i):
            raise ValueError(f"{n} cells cannot be halved {i} times")
        out.append(n // 2 ** i)
    return out


# ---------------------------------------------------------------- dense 1-D T
def cell_T_matrix(n_coarse):
    """Dense cell-based interpolation matrix, shape (2n, n) (Section 2.2)."""
    n = n_coarse
    if n < 2:
        raise ValueError("cell-based extrapolation needs at least 2 coarse cells")
    T = np.zeros((2 * n, n))
    for f in range(2 * n):
        J = f // 2
        if f == 0:
            T[f, 0], T[f, 1] = 1.25, -0.25
        elif f == 2 * n - 1:
            T[f, n - 1], T[f, n - 2] = 1.25, -0.25
        elif f % 2 == 0:          # left half of coarse cell J
            T[f, J], T[f, J - 1] = 0.75, 0.25
        else:                     # right half of coarse cell J
            T[f, J], T[f, J + 1] = 0.75, 0.25
    return T


def node_T_matrix(n_coarse_cells):
    """Dense node-based interpolation matrix, shape (2n+1, n+1) (Section 2.2)."""
    n = n_coarse_cells
    T = np.zeros((2 * n + 1, n + 1))
    for f in range(2 * n + 1):
        if f % 2 == 0:
            T[f, f // 2] = 1.0
        else:
            T[f, f // 2] = 0.5
            T[f, f // 2 + 1] = 0.5
    return T


# ------------------------------------------------------ slicing forms of T, T^T
def _mv(x, axis):
    return torch.movedim(x, axis, 0)


def prolong_axis(c, axis, centering="cell"):
    """Apply the 1-D interpolation T along one axis of a tensor."""
    x = _mv(c, axis)
    n = x.shape[0]
    if centering == "cell":
        if n < 2:
            raise ValueError("cell-based extrapolation needs at least 2 coarse cells")
        out = torch.empty((2 * n,) + tuple(x.shape[1:]), dtype=x.dtype)
        # even fine cell 2J: 3/4 c[J] + 1/4 c[J-1]; odd 2J+1: 3/4 c[J] + 1/4 c[J+1]
        out[2::2] = 0.75 * x[1:] + 0.25 * x[:-1]
        out[1:-1:2] = 0.75 * x[:-1] + 0.25 * x[1:]
        # end cells: linear extrapolation
        out[0] = 1.25 * x[0] - 0.25 * x[1]
        out[-1] = 1.25 * x[-1] - 0.25 * x[-2]
    elif centering == "node":
        m = n - 1
        out = torch.empty((2 * m + 1,) + tuple(x.shape[1:]), dtype=x.dtype)
        out[0::2] = x
        out[1::2] = 0.5 * (x[:-1] + x[1:])
    else:
        raise ValueError(centering)
    return torch.movedim(out, 0, axis)


def restrict_axis(g, axis, centering="cell"):
    """Apply T^T (exact transpose of prolong_axis) along one axis."""
    x = _mv(g, axis)
    nf = x.shape[0]
    if centering == "cell":
        n = nf // 2
        ev, od = x[0::2], x[1::2]           # fine cells 2J and 2J+1
        out = 0.75 * ev + 0.75 * od
        out = out.clone()
        out[1:] += 0.25 * od[:-1]           # fine 2J-1 -> coarse J (weight 1/4)
        out[:-1] += 0.25 * ev[1:]           # fine 2J+2 -> coarse J (weight 1/4)
        # end rows of T differ from the interior pattern
        out[0] += 0.5 * ev[0]               # 5/4 instead of 3/4
        out[1] -= 0.25 * ev[0]              # -1/4 on the neighbour
        out[n - 1] += 0.5 * od[n - 1]
        out[n - 2] -= 0.25 * od[n - 1]
    elif centering == "node":
        m = (nf - 1) // 2
        out = x[0::2].clone()
        out[:-1] += 0.5 * x[1::2]
        out[1:] += 0.5 * x[1::2]
        assert out.shape[0] == m + 1
    else:
        raise ValueError(centering)
    return torch.movedim(out, 0, axis)


def prolong(c, axes, centering="cell"):
    """Tensor-product interpolation T along every axis in `axes`."""
    for a in axes:
        c = prolong_axis(c, a, centering)
    return c


def restrict(g, axes, centering="cell"):
    """Transpose of prolong (T^T along every axis in `axes`)."""
    for a in axes:
        g = restrict_axis(g, a, centering)
    return g


# --------------------------------------------------------------- M_L and M_L^T
def decompose_horner(levels, axes, centering="cell"):
    """M_L(u_1..u_L) in Horner form, u_1 + T_1(u_2 + T_2(... + T_{L-1} u_L))."""
    w = levels[-1]
    for lvl in reversed(levels[:-1]):
        w = lvl + prolong(w, axes, centering)
    return w


def decompose_direct(levels, axes, centering="cell"):
    """M_L(u_1..u_L) as the direct sum u_1 + T_1 u_2 + T_1 T_2 u_3 + ..."""
    total = levels[0].clone()
    for i in range(1, len(levels)):
        x = levels[i]
        for _ in range(i):
            x = prolong(x, axes, centering)
        total = total + x
    return total


def decompose_transpose(g, n_levels, axes, centering="cell"):
    """M_L^T g: one field per level, (M^T g)_l = T_{l-1}^T ... T_1^T g."""
    out = [g]
    for _ in range(1, n_levels):
        out.append(restrict(out[-1], axes, centering))
    return out


def dense_decomposition_matrix(n, n_levels, ndim, centering="cell"):
    """Dense matrix of M_L for a d-dimensional field (tiny grids only).

    Built from Kronecker products of the dense 1-D matrices; columns are
    ordered level by level, each level in C order.
    """
    blocks = []
    if centering == "cell":
        sizes = level_sizes(n, n_levels)
        one_d = [np.eye(n)]
        for i in range(1, n_levels):
            one_d.append(one_d[-1] @ cell_T_matrix(sizes[i]))
    else:
        sizes = level_sizes(n, n_levels)
        one_d = [np.eye(n + 1)]
        for i in range(1, n_levels):
            one_d.append(one_d[-1] @ node_T_matrix(sizes[i]))
    for P in one_d:
        K = np.ones((1, 1))
        for _ in range(ndim):
            K = np.kron(K, P)
        blocks.append(K)
    return np.concatenate(blocks, axis=1)
