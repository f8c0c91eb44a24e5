"""Small oracle problem instances shared by the CPU and GPU tests.

Each builder returns an oracle Spec plus the list-of-levels shapes; inputs
are drawn from the seeded synthetic-input module.
"""
import math

import numpy as np

from oracle import operators as ops
from paper_2303_04679_amd import synth

NS_PARAMS = {"re": 60.0, "diam": 0.4, "lam": 1.0, "chi_shift": 5.0, "tau_coef": 0.5}


def _meas(seed, dims, n, field, term, weight, lo=None, hi=None):
    idx = synth.unique_cells(seed, dims, lo, hi, n)
    vals = synth.rng(seed + 1).uniform(-1, 1, size=n)
    return (field, term, idx, vals, weight)


def case(op, dims, n_levels, seed=0, with_forcing=False):
    """A random instance of `op` on `dims` with every loss term switched on."""
    dims = tuple(dims)
    nd = len(dims)
    if op == "poisson":
        spec = ops.Spec("poisson", dims, (1.0,) * nd, n_levels, weights={"pde": 1.0})
        spec.forcing = {0: synth.rng(seed + 5).uniform(-50, 50, size=dims)}
        return spec
    if op == "poisson_node":
        spec = ops.Spec("poisson", dims, (1.0,) * nd, n_levels, weights={"pde": 1.0, "bc": 1.0},
                        centering="node")
        spec.forcing = {0: synth.rng(seed + 5).uniform(-50, 50, size=tuple(d + 1 for d in dims))}
        return spec
    if op == "burgers":
        spec = ops.Spec("burgers", dims, (1.0, 2.0), n_levels,
                        weights={"pde": 1.0, "data": 100.0, "reg": 1e-4})
        n = max(2, min(32, dims[0] * dims[1] // 8))
        spec.meas = [_meas(seed + 11, dims, n, 0, "data", 100.0 / n, (1, 1), (dims[0] - 1, dims[1] - 1))]
    elif op == "heat":
        spec = ops.Spec("heat", dims, (0.02, 1.0), n_levels,
                        weights={"pde": 1.0, "data": 1.0, "ic": 1.0, "bc": 1.0})
        n = max(2, min(200, dims[0] * dims[1] // 8))
        x = synth.cell_centres(dims[1], 0.0, 1.0)
        spec.meas = [_meas(seed + 11, dims, n, 0, "data", 1.0 / n, (1, 0), dims),
                     (0, "ic", np.arange(dims[1], dtype=np.int32), synth.heat_initial(x), 1.0 / dims[1])]
    elif op in ("ns3d", "ns3d_fixed"):
        spec = ops.Spec(op, dims, (1.0, 1.0, 1.0), n_levels, params=dict(NS_PARAMS),
                        weights={"pde": 1.0, "data": 1.0})
        plane = synth.wake_plane_cells(dims)
        n = plane.size
        g = synth.rng(seed + 21)
        spec.meas = [(c, "data", plane, g.uniform(-1, 1, size=n), 1.0 / n) for c in range(3)]
        if op == "ns3d_fixed":
            spec.chi = synth.rng(seed + 31).uniform(0, 1, size=dims)
    elif op in ("ns3d_node", "ns3d_fixed_node"):
        base = op[:-5]
        spec = ops.Spec(base, dims, (1.0, 1.0, 2.0), n_levels,
                        params=dict(NS_PARAMS, u_ref=0.8),
                        weights={"pde": 1.0, "data": 1.0}, centering="node")
        shape = tuple(d + 1 for d in dims)
        n = max(2, min(96, math.prod(dims) // 16))
        # interior nodes only (the boundary nodes carry imposed values)
        idx = synth.unique_cells(seed + 21, shape, lo=(1,) * 3, hi=dims, n=n)
        g = synth.rng(seed + 22)
        spec.meas = [(c, "data", idx, g.uniform(-1, 1, size=n), 1.0 / n) for c in range(3)]
        if base == "ns3d_fixed":
            spec.chi = synth.rng(seed + 31).uniform(0, 1, size=shape)
    elif op in ("cavity", "cavity_node"):
        node = op == "cavity_node"
        spec = ops.Spec("cavity", dims, (1.0, 1.0), n_levels,
                        params={"re": 400.0, "tau_coef": 0.5, "u_ref": 1.0},
                        weights={"pde": 1.0, "data": 1.0}, centering="node" if node else "cell")
        shape = tuple(d + 1 for d in dims) if node else dims
        n = max(2, min(64, dims[0] * dims[1] // 8))
        # node-based: measure interior nodes only (the wall nodes carry imposed values)
        lo, hi = ((1,) * 2, dims) if node else (None, None)
        idx = synth.unique_cells(seed + 41, shape, lo=lo, hi=hi, n=n)
        g = synth.rng(seed + 42)
        spec.meas = [(c, "data", idx, g.uniform(-1, 1, size=n), 1.0 / n) for c in range(2)]
    else:
        raise ValueError(op)
    if with_forcing:
        neq = {"burgers": 1, "heat": 1, "ns3d": 4, "ns3d_fixed": 4, "ns3d_node": 4,
               "ns3d_fixed_node": 4, "cavity": 3, "cavity_node": 3}[op]
        g = synth.rng(seed + 51)
        shape = tuple(d + 1 for d in dims) if spec.centering == "node" else dims
        spec.forcing = {e: g.uniform(-1, 1, size=shape) for e in range(neq)}
    return spec


def random_levels(spec, seed, lo=-1.0, hi=1.0):
    shapes = ops.level_shapes(spec.op, spec.dims, spec.n_levels, spec.centering)
    return synth.uniform_levels(shapes, seed, lo, hi)
