"""Pins of the oracle's L-BFGS (Nocedal & Wright's limited-memory BFGS with a
strong-Wolfe line search; the paper's optimiser in Sections 2.1, 3.1, 3.3).

* the two-loop recursion equals the dense inverse-BFGS matrix built by the
  rank-two update formula applied pair by pair to gamma I (brute force)
* every accepted step satisfies the strong Wolfe conditions
* the minimiser matches scipy.optimize's L-BFGS-B (a library routine) on a
  smooth test function, and the iteration reaches the exact discrete
  solution of the manufactured Poisson problem through the multigrid
  decomposition, as the paper reports for L-BFGS (Section 3.1)
"""
import math

import numpy as np
import pytest
import scipy.optimize
import torch

from oracle import lbfgs as ol
from oracle import multigrid as mg
from oracle import operators as ops
from oracle import reference as ref


def _pairs(n, k, seed):
    """k random pairs with positive curvature s^T y > 0 (y = A s, A SPD)."""
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    S = [rng.standard_normal(n) for _ in range(k)]
    Y = [A @ s + 0.1 * rng.standard_normal(n) for s in S]
    for s, y in zip(S, Y):
        assert s @ y > 0
    return S, Y


def _dense_h(S, Y):
    n = S[0].size
    s, y = S[-1], Y[-1]
    H = (s @ y) / (y @ y) * np.eye(n)
    for s, y in zip(S, Y):
        rho = 1.0 / (y @ s)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


@pytest.mark.parametrize("k", [1, 2, 5, 9])
def test_two_loop_equals_dense_bfgs_matrix(k):
    S, Y = _pairs(12, k, seed=k)
    g = np.random.default_rng(100 + k).standard_normal(12)
    H = _dense_h(S, Y)
    got = ol.two_loop(g, S, Y)
    assert np.linalg.norm(got - H @ g) <= 1e-12 * np.linalg.norm(H @ g)


def test_two_loop_without_pairs_is_identity():
    g = np.arange(5.0)
    assert np.array_equal(ol.two_loop(g, [], []), g)


def test_cubic_step_is_exact_for_a_cubic():
    # phi(a) = (a - 1)^3 / 3 - (a - 1) + 7 has its local minimum at a = 2
    phi = lambda a: (a - 1) ** 3 / 3 - (a - 1) + 7
    dphi = lambda a: (a - 1) ** 2 - 1
    t = ol.cubic_step(1.5, phi(1.5), dphi(1.5), 3.0, phi(3.0), dphi(3.0))
    assert abs(t - 2.0) < 1e-12


def _rosenbrock(x):
    f = 100.0 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2
    g = np.array([-400.0 * x[0] * (x[1] - x[0] ** 2) - 2 * (1 - x[0]), 200.0 * (x[1] - x[0] ** 2)])
    return f, g


@pytest.mark.parametrize("x0,d,alpha1", [
    ((-1.2, 1.0), None, 1.0),      # steepest descent, first trial far too long: zoom
    ((-1.2, 1.0), None, 1e-6),     # first trial far too short: extrapolation
    ((0.5, 0.5), (1.0, 0.0), 1.0),
])
def test_line_search_satisfies_strong_wolfe(x0, d, alpha1):
    x = np.array(x0)
    f0, g0 = _rosenbrock(x)
    d = -g0 if d is None else np.array(d) * -np.sign(g0[0])
    dphi0 = float(g0 @ d)
    assert dphi0 < 0
    r = ol.line_search(_rosenbrock, x, d, f0, dphi0, alpha1)
    assert r.status == 0
    fa, ga = _rosenbrock(x + r.alpha * d)
    assert fa == r.f
    assert fa <= f0 + 1e-4 * r.alpha * dphi0
    assert abs(ga @ d) <= 0.9 * abs(dphi0)


def test_rosenbrock_minimum_and_scipy_agreement():
    it = ol.LBFGS(_rosenbrock, np.array([-1.2, 1.0]), m=10)
    for _ in range(200):
        if np.linalg.norm(it.g) < 1e-10:
            break
        it.step()
    assert np.linalg.norm(it.x - 1.0) < 1e-8
    sp = scipy.optimize.minimize(_rosenbrock, np.array([-1.2, 1.0]), jac=True, method="L-BFGS-B",
                                 options={"gtol": 1e-12, "ftol": 1e-16, "maxcor": 10})
    assert np.linalg.norm(it.x - sp.x) < 1e-5


def test_quadratic_matches_scipy_minimiser():
    rng = np.random.default_rng(7)
    n = 40
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    A = Q @ np.diag(np.logspace(0, 2, n)) @ Q.T
    b = rng.standard_normal(n)
    fg = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)
    it = ol.LBFGS(fg, np.zeros(n), m=8)
    for _ in range(300):
        if np.linalg.norm(it.g) < 1e-11 or it.step().status == 2:
            break
    # f is O(1) here, so comparing function values resolves x only to about
    # sqrt(eps) in the softest direction: the line search stops there
    exact = np.linalg.solve(A, b)
    assert np.linalg.norm(it.x - exact) < 1e-6 * np.linalg.norm(exact)
    sp = scipy.optimize.minimize(fg, np.zeros(n), jac=True, method="L-BFGS-B",
                                 options={"gtol": 1e-12, "ftol": 1e-20, "maxcor": 8})
    assert np.linalg.norm(it.x - sp.x) < 1e-6 * np.linalg.norm(exact)


def test_memory_keeps_the_newest_m_pairs():
    rng = np.random.default_rng(3)
    n = 20
    A = np.diag(np.linspace(1, 30, n))
    fg = lambda x: (0.5 * x @ A @ x, A @ x)
    it = ol.LBFGS(fg, rng.standard_normal(n), m=3)
    xs = []
    for _ in range(6):
        xs.append(it.x.copy())
        it.step()
    assert len(it.S) == 3
    assert np.allclose(it.S[-1], it.x - xs[-1], rtol=1e-12, atol=1e-15)


def _flat(levels):
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for row in levels for a in row])


def _unflat(x, shapes):
    out, o = [], 0
    for row in shapes:
        r = []
        for s in row:
            n = int(np.prod(s))
            r.append(x[o:o + n].reshape(s))
            o += n
        out.append(r)
    return out


@pytest.mark.parametrize("L", [1, 3])
def test_poisson_manufactured_solution_is_reached(L):
    """mODIL with L-BFGS on the 1-D cell-based Poisson problem reaches the exact
    discrete solution (the paper's Section 3.1 reports machine precision)."""
    n = 32
    spec = ops.Spec("poisson", (n,), (1.0,), L, weights={"pde": 1.0})
    u_ref = ref.poisson_reference((n,))
    spec.forcing = {0: ref.poisson_forcing(spec, u_ref)}
    shapes = ops.level_shapes("poisson", (n,), L)

    def fg(x):
        terms, grads = ops.loss_and_grad(spec, _unflat(x, shapes))
        return sum(terms.values()), _flat(grads)

    x0 = np.zeros(sum(int(np.prod(s)) for row in shapes for s in row))
    it = ol.LBFGS(fg, x0, m=50)
    for _ in range(400):
        if it.f < 1e-26:
            break
        ls = it.step()
        if ls.status == 2:
            break
    lv = [[torch.as_tensor(a) for a in row] for row in _unflat(it.x, shapes)]
    fine = ops.fine_fields(spec, lv)[0].detach().numpy()
    assert np.max(np.abs(fine - u_ref)) < 1e-8
