"""Forward solvers and closed forms that produce reference fields.

These generate the data that the inverse problems are posed on, the way the
paper does: the reference field is the solution of the discrete forward
problem (Sections 3.1, 3.2, 3.4).  Random draws (amplitudes, measurement
cells, noise) are inputs.
"""
import math

import numpy as np
import torch

from . import operators


def poisson_reference(dims):
    """u_ref(x) = g(prod_i 5(1 - x_i) x_i), g(v) = (v^5 / (1 + v^5))^(1/5) (Section 3.1)."""
    grids = np.meshgrid(*[(np.arange(n) + 0.5) / n for n in dims], indexing="ij")
    v = np.ones(dims)
    for x in grids:
        v = v * 5.0 * (1.0 - x) * x
    return (v ** 5 / (1.0 + v ** 5)) ** 0.2


def poisson_forcing(spec, u_ref):
    """f := discrete Laplacian of u_ref, so u_ref solves the discrete problem exactly."""
    s = operators.Spec("poisson", spec.dims, spec.lengths, 1)
    with torch.no_grad():
        R = operators.poisson_residual(s, torch.as_tensor(u_ref, dtype=torch.float64))[0]
    return R.numpy()


def _burgers_row_residual(un, uprev, dt, dx):
    F = 0.25 * (un[:-1] ** 2 + un[1:] ** 2) - 0.5 * np.abs(0.5 * (un[:-1] + un[1:])) * (un[1:] - un[:-1])
    flux = np.concatenate([[0.0], F, [0.0]])        # closed walls: zero boundary flux
    return (un - uprev) / dt + (flux[1:] - flux[:-1]) / dx


def burgers_forward(u0, n_rows, dt, dx, tol=1e-14, max_newton=50):
    """March the implicit upwind scheme from the initial row u0.

    Each row solves the same residual as the loss at every cell, with zero
    flux through the two walls, by Newton's method.  Returns (n_rows, N).
    """
    N = u0.shape[0]
    out = np.zeros((n_rows, N))
    out[0] = u0
    for n in range(1, n_rows):
        prev = out[n - 1]
        x = prev.copy()
        for _ in range(max_newton):
            r = _burgers_row_residual(x, prev, dt, dx)
            J = np.zeros((N, N))
            eps = 1e-7
            # Jacobian by columns; each column is a perturbed residual
            for j in range(N):
                xp = x.copy()
                xp[j] += eps
                xm = x.copy()
                xm[j] -= eps
                J[:, j] = (_burgers_row_residual(xp, prev, dt, dx)
                           - _burgers_row_residual(xm, prev, dt, dx)) / (2 * eps)
            dx_ = np.linalg.solve(J, -r)
            x = x + dx_
            if np.max(np.abs(dx_)) < tol * max(1.0, np.max(np.abs(x))):
                break
        out[n] = x
    return out


def heat_ic(x):
    """Initial temperature u(x, 0) = g(x) - g(0), g(x) = exp(-50 (x - 0.5)^2) (Section 3.4)."""
    g = lambda s: np.exp(-50.0 * (s - 0.5) ** 2)
    return g(x) - g(0.0)


def heat_forward(u0, k, n_rows, dt, dx):
    """Solve the implicit heat scheme row by row for a given cell conductivity k.

    Inner cells use the same residual as the loss; the two end rows impose the
    quadratic-extrapolated wall value zero.  Returns (n_rows, N).
    """
    N = u0.shape[0]
    out = np.zeros((n_rows, N))
    out[0] = u0
    kp = 0.5 * (k[1:-1] + k[2:])
    km = 0.5 * (k[1:-1] + k[:-2])
    A = np.zeros((N, N))
    A[0, 0:3] = [15 / 8, -10 / 8, 3 / 8]
    A[N - 1, N - 3:] = [3 / 8, -10 / 8, 15 / 8]
    for i in range(1, N - 1):
        A[i, i - 1] = -km[i - 1] / dx ** 2
        A[i, i] = 1.0 / dt + (kp[i - 1] + km[i - 1]) / dx ** 2
        A[i, i + 1] = -kp[i - 1] / dx ** 2
    for n in range(1, n_rows):
        b = np.zeros(N)
        b[1:-1] = out[n - 1, 1:-1] / dt
        out[n] = np.linalg.solve(A, b)
    return out


def inverse_softplus(k):
    """q with softplus(q) = k, for k > 0."""
    k = np.asarray(k, dtype=np.float64)
    return np.where(k > 30.0, k, np.log(np.expm1(np.minimum(k, 30.0))))
