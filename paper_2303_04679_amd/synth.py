"""Seeded synthetic inputs for the mODIL problems.

This module only draws random numbers and evaluates problem inputs (initial
conditions, conductivity profiles, body shapes, measurement locations).  It
holds none of the method's arithmetic (no interpolation, residual, gradient or
optimiser), so that both the HIP path and the independent CPU reference can
take their inputs from it.  Every function takes an explicit seed and uses
numpy.random.default_rng.
"""
import numpy as np


def rng(seed):
    return np.random.default_rng(seed)


def uniform_levels(shapes, seed, lo=-1.0, hi=1.0):
    """Random level fields: shapes is a list over levels of list of field shapes."""
    g = rng(seed)
    return [[g.uniform(lo, hi, size=s) for s in row] for row in shapes]


def unique_cells(seed, dims, lo=None, hi=None, n=1):
    """n distinct cells drawn uniformly from the box lo <= idx < hi; flat C-order indices, sorted."""
    dims = tuple(int(d) for d in dims)
    lo = tuple(lo) if lo is not None else (0,) * len(dims)
    hi = tuple(hi) if hi is not None else dims
    box = [h - l for l, h in zip(lo, hi)]
    total = int(np.prod(box))
    if n > total:
        raise ValueError("more cells requested than the box holds")
    pick = rng(seed).choice(total, size=n, replace=False)
    sub = np.unravel_index(pick, box)
    full = tuple(s + l for s, l in zip(sub, lo))
    return np.sort(np.ravel_multi_index(full, dims)).astype(np.int32)


def cell_centres(n, x0, x1):
    h = (x1 - x0) / n
    return x0 + (np.arange(n) + 0.5) * h


# ------------------------------------------------------------------- Burgers
def burgers_amplitudes(seed, count=3):
    """Amplitudes of the initial sinusoids, U(-0.5, 0.5)."""
    return rng(seed).uniform(-0.5, 0.5, size=count)


def burgers_ic(x, amps):
    """u(x, 0) = sum_k a_k sin(k pi x), k = 1..len(amps), on x in [-1, 1]."""
    return sum(a * np.sin((k + 1) * np.pi * x) for k, a in enumerate(amps))


# ---------------------------------------------------------------------- heat
def heat_conductivity(x, seed):
    """k(x) = 1 + 0.5 exp(-(x - c)^2 / (2 s^2)), c ~ U(0.3, 0.7), s ~ U(0.05, 0.15)."""
    g = rng(seed)
    c = g.uniform(0.3, 0.7)
    s = g.uniform(0.05, 0.15)
    return 1.0 + 0.5 * np.exp(-((x - c) ** 2) / (2.0 * s * s))


def gaussian_noise(seed, n, sigma):
    return rng(seed).normal(0.0, sigma, size=n)


def heat_initial(x):
    """Initial temperature g(x) - g(0), g(x) = exp(-50 (x - 0.5)^2)."""
    return np.exp(-50.0 * (x - 0.5) ** 2) - np.exp(-50.0 * 0.25)


# ------------------------------------------------------------ body in channel
def ellipsoid_axes(seed):
    """Semi-axes of the body, each U(0.15, 0.3) of the unit domain."""
    return rng(seed).uniform(0.15, 0.3, size=3)


def ellipsoid_chi(dims, axes, centre=(0.4, 0.5, 0.5)):
    """Sharp body fraction on a (z, y, x) cell grid over [0, 1]^3: 1 inside the ellipsoid."""
    nz, ny, nx = dims
    z = cell_centres(nz, 0.0, 1.0)[:, None, None]
    y = cell_centres(ny, 0.0, 1.0)[None, :, None]
    x = cell_centres(nx, 0.0, 1.0)[None, None, :]
    ax, ay, az = axes
    cx, cy, cz = centre
    r = ((x - cx) / ax) ** 2 + ((y - cy) / ay) ** 2 + ((z - cz) / az) ** 2
    return (r <= 1.0).astype(np.float64)


def wake_plane_cells(dims, frac=0.85):
    """All cells of the x-plane at index floor(frac * Nx), flat C-order (z, y, x)."""
    nz, ny, nx = dims
    i = int(np.floor(frac * nx))
    zz, yy = np.meshgrid(np.arange(nz), np.arange(ny), indexing="ij")
    return np.sort(np.ravel_multi_index((zz.ravel(), yy.ravel(), np.full(zz.size, i)),
                                        dims)).astype(np.int32)


# -------------------------------------------------------------------- cavity
def cavity_reynolds(seed):
    """Reynolds number of one cavity instance, U(100, 1000)."""
    return float(rng(seed).uniform(100.0, 1000.0))


def cavity_points(seed, dims, n=64):
    return unique_cells(seed + 7_000_000, dims, n=n)
