"""The benchmark workloads, as ProblemSpec + seeded synthetic inputs.

  burgers64    1-D inviscid Burgers, space-time 64 x 64, x in [-1, 1], t in
               [0, 1], FP64, levels 64..4 (L = 5), data at 32 random inner
               cells (weight 1e2 / 32), smoothing weight 1e-4
  heat256      heat conduction with unknown k(x) = softplus(q), 256 x 256,
               t in [0, 0.02], FP64 or FP32, L = 6 for u and q, initial
               condition on row 0, data at 200 random cells
  ns3d64       channel flow past an ellipsoid, 64^3, FP32, L = 5, unknown
               u, v, w, p, chihat; velocity measured on the wake plane
  ns3d128      the same at 128^3, L = 6
  ns3d256      the same at 256^3, L = 7 (2.3 GB per iteration, beyond the
               256 MB last-level cache)
  ns3d128_shard8  one GPU's share of ns3d128 split in z-slabs over eight
               GPUs: 16 x 128 x 128 cells at the same spacing, L = 4 (the
               levels a slab keeps; the coarser ones would be replicated);
               its z faces are walls here, where a rank would have halos
  cavity128    lid-driven cavity, 128 x 128, FP32, L = 5, Re ~ U(100, 1000),
               velocity at 64 random cells
  channel_node129  the channel of the body-shape study on its node grid:
               129 x 65 x 65 nodes over [0, 2] x [0, 1] x [0, 1] (h = 1/64),
               FP32, L = 6, unknown u, v, w, p, chihat; velocity at a
               19 x 6 x 6 lattice of nodes (684 points)

Measured values are seeded synthetic numbers of the magnitude of the
solution (the throughput of one iteration does not depend on them); the
reconstruction drivers replace them by values from a forward solve.
"""
import dataclasses

import numpy as np

from . import synth
from .modil import ProblemSpec


@dataclasses.dataclass
class Workload:
    name: str
    spec: ProblemSpec
    meas: list           # (instance, field, term, idx, values, weight)
    init: dict           # field name -> constant initial value on the coarsest level
    lr: float
    iterations: int
    chi: np.ndarray = None


def burgers64(seed=1):
    spec = ProblemSpec("burgers", (64, 64), (1.0, 2.0), 5, dtype="f64", max_meas=32,
                       w_pde=1.0, w_reg=1e-4)
    amps = synth.burgers_amplitudes(seed)
    idx = synth.unique_cells(seed + 1, (64, 64), (1, 1), (63, 63), 32)
    x = synth.cell_centres(64, -1.0, 1.0)[idx % 64]
    vals = synth.burgers_ic(x, amps)
    return Workload("burgers64", spec, [(0, 0, "data", idx, vals, 100.0 / 32)], {}, 1e-3, 2000)


def heat256(dtype="f64", seed=3):
    n = 256
    spec = ProblemSpec("heat", (n, n), (0.02, 1.0), 6, dtype=dtype, max_meas=200 + n,
                       w_pde=1.0, w_bc=1.0)
    x = synth.cell_centres(n, 0.0, 1.0)
    u0 = synth.heat_initial(x)
    idx = synth.unique_cells(seed + 1, (n, n), (1, 0), (n, n), 200)
    noise = synth.gaussian_noise(seed + 2, 200, 0.01 * np.max(np.abs(u0)))
    vals = u0[idx % n] * 0.9 + noise
    meas = [(0, 0, "ic", np.arange(n, dtype=np.int32), u0, 1.0 / n),
            (0, 0, "data", idx, vals, 1.0 / 200)]
    return Workload("heat256", spec, meas, {"q": float(np.log(np.e - 1.0))}, 1e-3, 5000)


def ns3d(n=128, levels=6, seed=6, dtype="f32"):
    spec = ProblemSpec("ns3d", (n, n, n), (1.0, 1.0, 1.0), levels, dtype=dtype,
                       max_meas=3 * n * n, re=60.0, diam=0.4, lam=1.0, chi_shift=5.0,
                       tau_coef=0.5, u_ref=1.0, w_pde=1.0)
    plane = synth.wake_plane_cells((n, n, n))
    g = synth.rng(seed + 100)
    meas = []
    for c, (mean, spread) in enumerate(((1.0, 0.1), (0.0, 0.05), (0.0, 0.05))):
        vals = mean + spread * g.standard_normal(plane.size)
        meas.append((0, c, "data", plane, vals, 1.0 / plane.size))
    chi = synth.ellipsoid_chi((n, n, n), synth.ellipsoid_axes(seed))
    return Workload(f"ns3d{n}", spec, meas, {"u": 1.0}, 1e-3, 3000, chi=chi)


def ns3d_shard(n=128, ranks=8, levels=4, seed=6, dtype="f32"):
    nz = n // ranks
    spec = ProblemSpec("ns3d", (nz, n, n), (nz / n, 1.0, 1.0), levels, dtype=dtype,
                       max_meas=3 * nz * n, re=60.0, diam=0.4, lam=1.0, chi_shift=5.0,
                       tau_coef=0.5, u_ref=1.0, w_pde=1.0)
    plane = synth.wake_plane_cells((nz, n, n))
    g = synth.rng(seed + 100)
    meas = []
    for c, (mean, spread) in enumerate(((1.0, 0.1), (0.0, 0.05), (0.0, 0.05))):
        vals = mean + spread * g.standard_normal(plane.size)
        meas.append((0, c, "data", plane, vals, 1.0 / (n * n)))
    return Workload(f"ns3d{n}_shard{ranks}", spec, meas, {"u": 1.0}, 1e-3, 3000)


def channel_node_lattice(dims, m=6):
    """Flat node indices [z][y][x] of a lattice of 19 x-positions (x = 0.1 ..
    1.9) times m x m evenly spaced (y, z) positions, each at its nearest node;
    dims are cells (z, y, x) of [0, 1] x [0, 1] x [0, 2]."""
    nz, ny, nx = dims
    h = 2.0 / nx
    ys = (np.arange(m) + 0.5) / m
    out = [(int(round(z / h)) * (ny + 1) + int(round(y / h))) * (nx + 1) + int(round(x / h))
           for x in 0.1 * np.arange(1, 20) for y in ys for z in ys]
    out = np.array(out, dtype=np.int32)
    assert np.unique(out).size == out.size
    return np.sort(out)


def channel_node129(seed=6, dtype="f32"):
    dims = (64, 64, 128)
    pts = channel_node_lattice(dims)
    spec = ProblemSpec("ns3d", dims, (1.0, 1.0, 2.0), 6, dtype=dtype, max_meas=3 * pts.size,
                       re=60.0, diam=0.4, lam=1.0, chi_shift=5.0, tau_coef=0.5, u_ref=1.0,
                       w_pde=1.0, centering="node")
    g = synth.rng(seed + 100)
    meas = []
    for c, (mean, spread) in enumerate(((1.0, 0.1), (0.0, 0.05), (0.0, 0.05))):
        vals = mean + spread * g.standard_normal(pts.size)
        meas.append((0, c, "data", pts, vals, 1.0 / pts.size))
    return Workload("channel_node129", spec, meas, {"u": 1.0}, 1e-3, 20000)


def cavity128(batch=1, seed=0):
    n = 128
    spec = ProblemSpec("cavity", (n, n), (1.0, 1.0), 5, dtype="f32", batch=batch,
                       max_meas=batch * 2 * 64, re=synth.cavity_reynolds(seed), w_pde=1.0)
    meas = []
    for b in range(batch):
        idx = synth.cavity_points(seed + b, (n, n))
        g = synth.rng(seed + b + 200)
        for c in range(2):
            meas.append((b, c, "data", idx, 0.2 * g.standard_normal(idx.size), 1.0 / idx.size))
    return Workload("cavity128", spec, meas, {}, 1e-3, 50000)


WORKLOADS = {
    "burgers64": burgers64,
    "heat256": heat256,
    "heat256_f32": lambda: heat256("f32"),
    "ns3d64": lambda: ns3d(64, 5),
    "ns3d128": lambda: ns3d(128, 6),
    "ns3d256": lambda: ns3d(256, 7),
    "ns3d128_shard8": lambda: ns3d_shard(128, 8, 4),
    "cavity128": cavity128,
    "channel_node129": channel_node129,
}


def build(workload, device="cuda"):
    """Context and an initial parameter pack for a Workload."""
    import torch

    from .modil import Context
    ctx = Context(workload.spec, device=device)
    for inst, field, term, idx, vals, w in workload.meas:
        ctx.set_measurements(field, idx, vals, w, term=term, instance=inst)
    if workload.spec.batch > 1 and workload.spec.op == "cavity":
        for b in range(workload.spec.batch):
            ctx.set_reynolds(b, synth.cavity_reynolds(b))
    theta = ctx.new_pack()
    names = list(workload.spec.fields)
    for b in range(workload.spec.batch):
        coarsest = ctx.level_views(theta, b)[-1]
        for name, value in workload.init.items():
            coarsest[names.index(name)].fill_(value)
    return ctx, theta
