"""Pins of the oracle's loss weighting, smoothing term and residual metric.

The PDE term of the loss is an integral of the squared residual (a sum over
the inner points times the cell measure, Sections 2.1 and 3.1), the Burgers
smoothing term an integral of the squared gradient over the inner faces
(Section 3.2), and the residual metric the RMS of the cell-integrated
residual.  States whose residual is a known constant (zero fields with a
constant forcing, the free stream with constant forcings) and fields linear in
x and t give these terms in closed form: a dropped or wrong cell measure, a
wrong count of inner points or faces, or a missing face direction changes the
value.
"""
import math

import numpy as np
import pytest

from oracle import operators as ops

NS = {"re": 60.0, "diam": 0.4, "lam": 1.0, "chi_shift": 5.0, "tau_coef": 0.5}


def _levels(spec, fine):
    """Level fields with `fine` (one array per field) on the finest level, zero below."""
    shapes = ops.level_shapes(spec.op, spec.dims, spec.n_levels, spec.centering)
    out = [[np.asarray(f, dtype=np.float64) for f in fine]]
    out += [[np.zeros(s) for s in row] for row in shapes[1:]]
    return out


@pytest.mark.parametrize("dims,lengths", [((12,), (0.7,)), ((8, 12), (0.5, 2.0)),
                                          ((4, 8, 6), (0.5, 1.5, 2.5))])
def test_poisson_pde_term_is_an_integral(dims, lengths):
    """u = 0 with constant forcing c: R = -c in every cell (the zero field
    satisfies the ghost rule), so the PDE term is w c^2 times the volume of
    the box, whatever the number of cells."""
    c, w = 3.0, 0.7
    spec = ops.Spec("poisson", dims, lengths, 2, weights={"pde": w})
    spec.forcing = {0: np.full(dims, c)}
    terms = ops.loss_value(spec, _levels(spec, [np.zeros(dims)]))
    assert terms["pde"] == pytest.approx(w * c * c * math.prod(lengths), rel=1e-14)
    # halving the cell size leaves the integral unchanged
    dims2 = tuple(2 * n for n in dims)
    spec2 = ops.Spec("poisson", dims2, lengths, 2, weights={"pde": w})
    spec2.forcing = {0: np.full(dims2, c)}
    terms2 = ops.loss_value(spec2, _levels(spec2, [np.zeros(dims2)]))
    assert terms2["pde"] == pytest.approx(terms["pde"], rel=1e-14)


@pytest.mark.parametrize("dims,lengths", [((12,), (0.7,)), ((8, 12), (0.5, 2.0)),
                                          ((4, 8, 6), (0.5, 1.5, 2.5))])
def test_poisson_node_pde_term_counts_interior_nodes(dims, lengths):
    """Node-based: the interior nodes carry the equations, each weighted by
    the cell measure h^d: w c^2 h^d prod(N_a - 1)."""
    c, w = 2.0, 1.3
    shape = tuple(n + 1 for n in dims)
    spec = ops.Spec("poisson", dims, lengths, 2, weights={"pde": w}, centering="node")
    spec.forcing = {0: np.full(shape, c)}
    terms = ops.loss_value(spec, _levels(spec, [np.zeros(shape)]))
    h = [L / n for L, n in zip(lengths, dims)]
    expect = w * c * c * math.prod(h) * math.prod(n - 1 for n in dims)
    assert terms["pde"] == pytest.approx(expect, rel=1e-14)


def test_ns3d_free_stream_with_forcing_is_an_integral():
    """The free stream (1, 0, 0), p = 0 without body is an exact discrete
    solution, so constant forcings f_e leave residuals -f_e in every cell:
    the PDE term is w |Omega| sum_e f_e^2 on a box of any shape."""
    dims, lengths = (4, 6, 8), (0.5, 0.75, 2.0)
    f = [0.3, -1.1, 0.7, 2.0]
    w = 0.9
    spec = ops.Spec("ns3d_fixed", dims, lengths, 2, params=dict(NS), weights={"pde": w},
                    chi=np.zeros(dims))
    spec.forcing = {e: np.full(dims, f[e]) for e in range(4)}
    z = np.zeros(dims)
    terms = ops.loss_value(spec, _levels(spec, [z + 1.0, z, z, z]))
    expect = w * math.prod(lengths) * sum(x * x for x in f)
    assert terms["pde"] == pytest.approx(expect, rel=1e-13)


@pytest.mark.parametrize("op", ["burgers", "heat"])
def test_space_time_pde_term_counts_inner_points(op):
    """Burgers and heat: a constant state has zero residual (any conductivity),
    so a constant forcing f leaves -f on the inner points n >= 1, 1 <= i <= N-2:
    the PDE term is w dt dx f^2 (N_t - 1)(N_x - 2)."""
    nt, nx = 10, 14
    lengths = (0.3, 2.0)
    fval, w = 1.7, 0.6
    spec = ops.Spec(op, (nt, nx), lengths, 2, weights={"pde": w})
    spec.forcing = {0: np.full((nt, nx), fval)}
    fine = [np.full((nt, nx), 0.4)]
    if op == "heat":
        fine.append(np.linspace(-1.0, 1.0, nx))   # any conductivity profile
    terms = ops.loss_value(spec, _levels(spec, fine))
    dt, dx = lengths[0] / nt, lengths[1] / nx
    expect = w * dt * dx * fval * fval * (nt - 1) * (nx - 2)
    assert terms["pde"] == pytest.approx(expect, rel=1e-13)


def test_burgers_smoothing_of_a_linear_field():
    """u = a x + b t has u_x = a on every x-face and u_t = b on every t-face:
    the smoothing term is w dt dx (a^2 N_t (N_x - 1) + b^2 (N_t - 1) N_x)."""
    nt, nx = 6, 10
    lengths = (0.5, 2.0)
    a, b, w = 1.5, -0.8, 1e-4
    dt, dx = lengths[0] / nt, lengths[1] / nx
    t = np.arange(nt) * dt
    x = -1.0 + (np.arange(nx) + 0.5) * dx
    u = a * x[None, :] + b * t[:, None]
    spec = ops.Spec("burgers", (nt, nx), lengths, 2, weights={"reg": w})
    terms = ops.loss_value(spec, _levels(spec, [u]))
    expect = w * dt * dx * (a * a * nt * (nx - 1) + b * b * (nt - 1) * nx)
    assert terms["reg"] == pytest.approx(expect, rel=1e-12)
    # each direction alone
    for aa, bb in ((a, 0.0), (0.0, b)):
        u1 = aa * x[None, :] + bb * t[:, None]
        t1 = ops.loss_value(spec, _levels(spec, [u1]))
        e1 = w * dt * dx * (aa * aa * nt * (nx - 1) + bb * bb * (nt - 1) * nx)
        assert t1["reg"] == pytest.approx(e1, rel=1e-12)


@pytest.mark.parametrize("dims,lengths", [((12,), (0.7,)), ((8, 12), (0.5, 2.0)),
                                          ((4, 8, 6), (0.5, 1.5, 2.5))])
def test_residual_metric_of_a_constant_residual(dims, lengths):
    """u = 0 with constant forcing c: every cell-integrated residual is -V c,
    so the RMS is V |c|."""
    c = -4.0
    spec = ops.Spec("poisson", dims, lengths, 2, weights={"pde": 1.0})
    spec.forcing = {0: np.full(dims, c)}
    r = ops.residual_metric(spec, _levels(spec, [np.zeros(dims)]))
    V = math.prod(L / n for L, n in zip(lengths, dims))
    assert r == pytest.approx(V * abs(c), rel=1e-14)


def test_residual_metric_averages_over_equations():
    """Free stream with constant forcings f_e: the four integrated residuals
    are -V f_e in every cell, so r = V sqrt(sum_e f_e^2 / 4)."""
    dims, lengths = (4, 6, 8), (0.5, 0.75, 2.0)
    f = [0.3, -1.1, 0.7, 2.0]
    spec = ops.Spec("ns3d_fixed", dims, lengths, 2, params=dict(NS), weights={"pde": 1.0},
                    chi=np.zeros(dims))
    spec.forcing = {e: np.full(dims, f[e]) for e in range(4)}
    z = np.zeros(dims)
    r = ops.residual_metric(spec, _levels(spec, [z + 1.0, z, z, z]))
    V = math.prod(L / n for L, n in zip(lengths, dims))
    assert r == pytest.approx(V * math.sqrt(sum(x * x for x in f) / 4.0), rel=1e-13)


@pytest.mark.parametrize("op,dims", [("cavity", (8, 12)), ("ns3d", (4, 8, 6)), ("heat", (8, 6)),
                                     ("cavity_node", (8, 6))])
def test_data_only_loss_on_one_level(op, dims):
    """With every weight but the data weight at zero and one level (M is the
    identity), the loss is the weighted sum of squared misfits at the
    measured points and its gradient 2 w (u - y) there, zero elsewhere:
    brute force over the measurement list."""
    from tests.oracle_cases import case, random_levels
    spec = case(op, dims, 1, seed=3)
    spec.weights = {t: 0.0 for t in spec.weights}
    spec.weights["data"] = 1.0
    spec.meas = [m for m in spec.meas if m[1] == "data"]
    lv = random_levels(spec, 4)
    terms, grad = ops.loss_and_grad(spec, lv)
    loss = 0.0
    want = [np.zeros_like(np.asarray(x)) for x in lv[0]]
    for fi, _, idx, vals, wt in spec.meas:
        u = np.asarray(lv[0][fi]).reshape(-1)[np.asarray(idx)]
        loss += wt * float(((u - vals) ** 2).sum())
        want[fi].reshape(-1)[np.asarray(idx)] += 2.0 * wt * (u - vals)
    assert terms["pde"] == 0.0 and terms["reg"] == 0.0 and terms["bc"] == 0.0
    assert terms["data"] == pytest.approx(loss, rel=1e-14)
    for g, w in zip(grad[0], want):
        np.testing.assert_allclose(g, w, rtol=0, atol=1e-14)
