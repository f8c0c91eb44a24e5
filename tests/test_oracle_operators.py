"""Pins of the oracle's residuals and loss terms against closed forms.

Each check ties the discrete operators to something other than their own
formula: exactness on polynomials, exact discrete solutions (constant and
free-stream states), the order of consistency with the continuous PDE,
conservation, and the special values the paper states.
"""
import math

import numpy as np
import pytest
import torch

from oracle import operators as ops
from oracle import reference as ref

DT = torch.float64


def _centres(n, x0=0.0, x1=1.0):
    return x0 + (np.arange(n) + 0.5) * (x1 - x0) / n


# --------------------------------------------------------------------- Poisson
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_poisson_exact_on_quadratics(ndim):
    """u = prod x_a(1 - x_a) vanishes on the walls; the 3-point Laplacian and the
    quadratic-extrapolation ghost are exact for it, so R = 0 in every cell."""
    n = 8
    x = _centres(n)
    grids = np.meshgrid(*([x] * ndim), indexing="ij")
    q = [g * (1 - g) for g in grids]
    u = np.prod(q, axis=0)
    lap = np.zeros_like(u)
    for a in range(ndim):
        term = -2.0 * np.ones_like(u)
        for b in range(ndim):
            if b != a:
                term = term * q[b]
        lap += term
    spec = ops.Spec("poisson", (n,) * ndim, (1.0,) * ndim, 1, forcing={0: lap})
    R = ops.poisson_residual(spec, torch.tensor(u))[0].numpy()
    assert np.max(np.abs(R)) < 1e-11


def test_poisson_manufactured_is_exact_minimum():
    """f := A_h(u_ref) (Section 3.1): u_ref gives zero loss and zero gradient, and
    the least-squares minimiser of the linear residual is u_ref."""
    n = 8
    spec = ops.Spec("poisson", (n, n), (1.0, 1.0), 1, weights={"pde": 1.0})
    u_ref = ref.poisson_reference((n, n))
    spec.forcing = {0: ref.poisson_forcing(spec, u_ref)}
    terms, grads = ops.loss_and_grad(spec, [[u_ref]])
    assert terms["pde"] < 1e-26
    assert np.max(np.abs(grads[0][0])) < 1e-10
    # dense linear map u -> A_h u (columns are residuals of unit vectors, f = 0)
    s0 = ops.Spec("poisson", (n, n), (1.0, 1.0), 1)
    cols = []
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = 1.0
        cols.append(ops.poisson_residual(s0, torch.tensor(e.reshape(n, n)))[0].numpy().ravel())
    A = np.stack(cols, 1)
    sol = np.linalg.lstsq(A, spec.forcing[0].ravel(), rcond=None)[0]
    np.testing.assert_allclose(sol, u_ref.ravel(), rtol=0, atol=1e-12)
    assert u_ref.max() > 0.5           # the reference is not trivial


# --------------------------------------------------------------------- Burgers
def test_upwind_flux_picks_upwind_state():
    """The flux is f(left) for positive face speed and f(right) for negative."""
    a = torch.tensor([0.5, 1.0, -0.2, -1.0], dtype=DT)
    b = torch.tensor([0.7, 0.1, -0.6, 0.4], dtype=DT)
    F = ops._upwind_flux(a, b).numpy()
    mean = 0.5 * (a + b).numpy()
    expect = np.where(mean > 0, 0.5 * a.numpy() ** 2, 0.5 * b.numpy() ** 2)
    np.testing.assert_allclose(F, expect, rtol=1e-15)


def _burgers_spec(nt, nx, **kw):
    return ops.Spec("burgers", (nt, nx), (1.0, 2.0), 1, **kw)


def test_burgers_constant_state():
    spec = _burgers_spec(8, 8, weights={"pde": 1.0, "reg": 1e-4})
    u = torch.full((8, 8), 0.37, dtype=DT)
    assert float(ops.loss_terms(spec, [u])["pde"]) == 0.0
    assert float(ops.loss_terms(spec, [u])["reg"]) == 0.0


def _burgers_consistency_error(n):
    spec = _burgers_spec(n, n)
    dt, dx = spec.h
    t = np.arange(n)[:, None] * dt
    x = _centres(n, -1.0, 1.0)[None, :]
    u = 1.0 + 0.3 * np.sin(np.pi * x) + 0.2 * t           # positive: one upwind side
    exact = 0.2 + u * 0.3 * np.pi * np.cos(np.pi * x)        # u_t + u u_x
    R = ops.burgers_residual(spec, torch.tensor(u))[0].numpy()
    return np.max(np.abs(R - exact[1:, 1:-1]))


def test_burgers_first_order_consistency():
    """The implicit upwind residual approximates u_t + u u_x to first order."""
    e1, e2 = _burgers_consistency_error(32), _burgers_consistency_error(64)
    assert e2 < e1 and 1.7 < e1 / e2 < 2.3


def test_burgers_forward_reference():
    """The generated reference has zero inner residual and conserves sum_i u_i
    (zero flux through the walls)."""
    n = 16
    spec = _burgers_spec(n, n, weights={"pde": 1.0})
    x = _centres(n, -1.0, 1.0)
    u0 = 0.3 * np.sin(np.pi * x) - 0.2 * np.sin(2 * np.pi * x)
    U = ref.burgers_forward(u0, n, *spec.h)
    R = ops.burgers_residual(spec, torch.tensor(U))[0].numpy()
    assert np.max(np.abs(R)) < 1e-10
    sums = U.sum(1)
    assert np.max(np.abs(sums - sums[0])) < 1e-12


# ------------------------------------------------------------------------ heat
def _heat_spec(nt, nx, T=0.02, **kw):
    return ops.Spec("heat", (nt, nx), (T, 1.0), 1, **kw)


def test_heat_constant_state_any_conductivity():
    spec = _heat_spec(6, 8)
    q = torch.tensor(np.random.default_rng(0).standard_normal(8))
    u = torch.full((6, 8), -0.8, dtype=DT)
    R = ops.heat_residual(spec, u, q)[0]
    assert float(R.abs().max()) == 0.0


def test_heat_wall_extrapolation_exact_for_quadratics():
    """(15 u0 - 10 u1 + 3 u2) / 8 is the face value of any quadratic."""
    n = 8
    x = _centres(n)
    u = np.tile(2.0 + 3.0 * x - 5.0 * x ** 2, (3, 1))
    left, right = ops.heat_boundary(_heat_spec(3, n), torch.tensor(u))
    np.testing.assert_allclose(left.numpy(), 2.0, rtol=1e-14)
    np.testing.assert_allclose(right.numpy(), 2.0 + 3.0 - 5.0, rtol=1e-13)


def _heat_consistency_error(n):
    T = 0.5
    spec = _heat_spec(n, n, T=T)
    dt, dx = spec.h
    t = np.arange(n)[:, None] * dt
    x = _centres(n)[None, :]
    kx = 1.0 + 0.5 * np.sin(2 * x)
    q = ref.inverse_softplus(kx[0])
    u = np.exp(-t) * np.cos(3 * x)
    u_t = -u
    u_x = -3 * np.exp(-t) * np.sin(3 * x)
    u_xx = -9 * u
    k_x = np.cos(2 * x)
    exact = u_t - (k_x * u_x + kx * u_xx)
    R = ops.heat_residual(spec, torch.tensor(u), torch.tensor(q))[0].numpy()
    return np.max(np.abs(R - exact[1:, 1:-1]))


def test_heat_consistency():
    """Residual approximates u_t - (k u_x)_x (first order in t, second in x)."""
    e1, e2 = _heat_consistency_error(32), _heat_consistency_error(64)
    assert e2 < e1 and e1 / e2 > 1.7


def test_heat_forward_reference_loss_is_noise():
    """With the true conductivity and the forward solution, only the data noise remains."""
    n = 16
    x = _centres(n)
    k = 1.0 + 0.5 * np.exp(-((x - 0.5) ** 2) / (2 * 0.1 ** 2))
    spec = _heat_spec(n, n, weights={"pde": 1.0, "data": 1.0, "ic": 1.0, "bc": 1.0})
    dt, dx = spec.h
    u0 = ref.heat_ic(x)
    U = ref.heat_forward(u0, k, n, dt, dx)
    idx = np.array([20, 77, 130, 201])
    noise = np.array([0.01, -0.02, 0.005, 0.0])
    spec.meas = [(0, "data", idx, U.ravel()[idx] + noise, 1.0 / 4),
                 (0, "ic", np.arange(n), u0, dx)]
    q = ref.inverse_softplus(k)
    terms = ops.loss_value(spec, [[U, q]])
    assert abs(terms["data"] - np.sum(noise ** 2) / 4) < 1e-15
    assert terms["pde"] < 1e-20 and terms["bc"] < 1e-24 and terms["ic"] == 0.0


def test_softplus_stable_and_exact():
    q = torch.tensor([-800.0, -30.0, -1.0, 0.0, 1e-8, 2.0, 40.0, 900.0], dtype=DT)
    k = ops.softplus(q).numpy()
    expect = [math.log1p(math.exp(v)) if v < 30 else v + math.log1p(math.exp(-v)) for v in q.tolist()]
    np.testing.assert_allclose(k, expect, rtol=1e-15)
    qq = q.clone().requires_grad_(True)
    (g,) = torch.autograd.grad(ops.softplus(qq).sum(), qq)
    np.testing.assert_allclose(g.numpy(), torch.sigmoid(q).numpy(), rtol=1e-15)


# ------------------------------------------------------------------------ ns3d
def _ns_spec(n, chi=None, op="ns3d_fixed", **kw):
    params = {"re": 60.0, "diam": 0.4, "lam": 1.0, "chi_shift": 5.0, "tau_coef": 0.5}
    return ops.Spec(op, (n, n, n), (1.0, 1.0, 1.0), 1, params=params, chi=chi, **kw)


def test_ns3d_free_stream_is_exact():
    """Uniform flow (1, 0, 0), p = 0, no body satisfies every equation and ghost rule."""
    n = 6
    z = np.zeros((n, n, n))
    spec = _ns_spec(n, chi=z)
    R = ops.ns3d_residual(spec, [torch.tensor(z + 1), torch.tensor(z), torch.tensor(z), torch.tensor(z)])
    assert max(float(r.abs().max()) for r in R) == 0.0


def test_ns3d_brinkman_inside_body():
    """Inside the body (chi = 1) the momentum residual is the penalty lambda * u."""
    n = 5
    rng = np.random.default_rng(1)
    f = [torch.tensor(rng.standard_normal((n, n, n))) for _ in range(4)]
    spec = _ns_spec(n, chi=np.ones((n, n, n)))
    R = ops.ns3d_residual(spec, f)
    for c in range(3):
        np.testing.assert_allclose(R[1 + c].numpy(), f[c].numpy(), rtol=1e-15)


def test_ns3d_chi_transform_initial_value():
    """chihat = 0 gives chi = 1 / (1 + e^5), the initial body fraction of Section 3.5."""
    spec = _ns_spec(4, op="ns3d")
    chi = ops.ns3d_chi(spec, torch.zeros(1, dtype=DT))
    assert abs(float(chi) - 1.0 / (1.0 + math.exp(5.0))) < 1e-17


def _smooth_fields(n):
    x = _centres(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    Xt, Yt, Zt = (torch.tensor(a, requires_grad=True) for a in (X, Y, Z))
    u = 1.0 + 0.3 * torch.sin(2 * Xt) * torch.cos(Yt) + 0.1 * Zt
    v = 0.2 * torch.cos(Xt + Zt) * torch.sin(2 * Yt)
    w = 0.1 * torch.sin(Xt * Yt + Zt)
    p = 0.5 * torch.cos(Xt) * torch.sin(Zt) + 0.2 * Yt ** 2
    return (Xt, Yt, Zt), (u, v, w, p)


def _derivs(fn, coords):
    g = torch.autograd.grad(fn.sum(), coords, create_graph=True)
    h = []
    for a in range(3):
        if g[a].requires_grad:
            ha = torch.autograd.grad(g[a].sum(), coords[a], retain_graph=True, allow_unused=True)[0]
        else:
            ha = None
        h.append(torch.zeros_like(coords[a]) if ha is None else ha)
    return [x.detach().numpy() for x in g], [x.detach().numpy() for x in h]


def _ns_consistency_error(n, nu=0.4 / 60.0, tau=0.5):
    coords, (u, v, w, p) = _smooth_fields(n)
    du, hu = _derivs(u, coords)
    dv, hv = _derivs(v, coords)
    dw, hw = _derivs(w, coords)
    dp, hp = _derivs(p, coords)
    U = [x.detach().numpy() for x in (u, v, w)]
    h = 1.0 / n
    cont = du[0] + dv[1] + dw[2] - tau * h * sum(hp)
    mom = []
    for D, H, comp in ((du, hu, 0), (dv, hv, 1), (dw, hw, 2)):
        conv = U[0] * D[0] + U[1] * D[1] + U[2] * D[2]
        mom.append(conv + dp[comp] - nu * sum(H))
    spec = _ns_spec(n, chi=np.zeros((n, n, n)))
    R = ops.ns3d_residual(spec, [torch.tensor(x.detach().numpy()) for x in (u, v, w, p)])
    inner = (slice(1, -1),) * 3
    errs = [np.max(np.abs(R[0].numpy() - cont)[inner])]
    errs += [np.max(np.abs(R[1 + c].numpy() - mom[c])[inner]) for c in range(3)]
    return np.array(errs)


def test_ns3d_second_order_consistency():
    """Interior residuals approximate the PDE (with the h-scaled pressure
    stabilisation) to second order: central differences."""
    e1, e2 = _ns_consistency_error(12), _ns_consistency_error(24)
    assert np.all(e1 / e2 > 3.3), e1 / e2


def test_ns3d_inlet_ghost_linear_profile():
    """u = 1 + a x has face value 1 at the inlet: the inlet cells see the exact
    derivative a and a zero Laplacian."""
    n, a = 6, 0.7
    x = _centres(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    z = np.zeros_like(X)
    spec = _ns_spec(n, chi=z)
    u = 1.0 + a * X
    R = ops.ns3d_residual(spec, [torch.tensor(u), torch.tensor(z), torch.tensor(z), torch.tensor(z)])
    np.testing.assert_allclose(R[0].numpy()[:, :, 0], a, rtol=1e-13)
    np.testing.assert_allclose(R[1].numpy()[:, :, 0], u[:, :, 0] * a, rtol=1e-13)


# ---------------------------------------------------------------------- cavity
def test_cavity_lid_and_walls():
    """u = y has value 0 on the bottom wall and 1 on the lid: every row sees the
    exact derivative du/dy = 1 through the ghosts and a zero Laplacian."""
    n = 8
    y = _centres(n)
    Y = np.tile(y[:, None], (1, n))
    z = np.zeros((n, n))
    spec = ops.Spec("cavity", (n, n), (1.0, 1.0), 1, params={"re": 100.0, "tau_coef": 0.5})
    R = ops.cavity_residual(spec, [torch.tensor(Y), torch.tensor(z), torch.tensor(z)])
    # momentum_u = u u_x + v u_y + p_x - lap u / Re = 0 everywhere except x walls
    # (u = y does not vanish on the side walls; their ghosts add a Laplacian)
    assert float(R[1][:, 1:-1].abs().max()) < 1e-12
    np.testing.assert_allclose(R[0].numpy()[:, 1:-1], 0.0, atol=1e-12)


def test_cavity_pressure_gauge_invariance():
    """p enters only through differences: the loss is invariant under p -> p + c."""
    n = 8
    rng = np.random.default_rng(3)
    f = [rng.standard_normal((n, n)) for _ in range(3)]
    spec = ops.Spec("cavity", (n, n), (1.0, 1.0), 1, params={"re": 400.0, "tau_coef": 0.5},
                    weights={"pde": 1.0})
    a = ops.loss_value(spec, [f])["pde"]
    b = ops.loss_value(spec, [[f[0], f[1], f[2] + 3.25]])["pde"]
    assert abs(a - b) <= 1e-13 * a


# ------------------------------------------------------ node-based cavity
def _cavity_node_spec(n, re=100.0, tau=0.5, lid=0.0, forcing=None, ny=None):
    ny = ny or n
    return ops.Spec("cavity", (ny, n), (1.0, 1.0), 1,
                    params={"re": re, "tau_coef": tau, "u_ref": lid},
                    weights={"pde": 1.0}, centering="node", forcing=forcing or {})


def test_cavity_node_exact_for_products_of_quadratics():
    """With a resting lid, u = q(x) q(y) and v = q(x) q(y) / 2 (q(s) = s (1 - s))
    vanish on the walls and are quadratic along each axis, where central
    differences are exact; with constant pressure the node residuals are the
    continuous Navier-Stokes operators evaluated at the nodes."""
    n, ny = 8, 6
    nu = 1.0 / 100.0
    y, x = np.arange(ny + 1) / ny, np.arange(n + 1) / n
    Y, X = np.meshgrid(y, x, indexing="ij")
    qx, qy, dqx, dqy = X * (1 - X), Y * (1 - Y), 1 - 2 * X, 1 - 2 * Y
    u, v = qx * qy, 0.5 * qx * qy
    ux, uy = dqx * qy, qx * dqy
    lap_u = -2.0 * qy - 2.0 * qx
    f = {0: ux + 0.5 * uy,
         1: u * ux + v * uy - nu * lap_u,
         2: 0.5 * (u * ux + v * uy - nu * lap_u)}
    spec = _cavity_node_spec(n, ny=ny, forcing=f)
    R = ops.cavity_node_residual(spec, [torch.tensor(u), torch.tensor(v), torch.full_like(torch.tensor(u), 2.5)])
    for r in R:
        assert r.shape == (ny - 1, n - 1)
        assert float(r.abs().max()) < 1e-13


def test_cavity_node_lid_row():
    """u = y with the lid at u = 1: the imposed lid (last row) and bottom wall
    (u = 0) agree with u = y, so away from the side walls every residual is zero."""
    n = 8
    y = np.arange(n + 1) / n
    Y = np.tile(y[:, None], (1, n + 1))
    z = np.zeros_like(Y)
    rng = np.random.default_rng(5)
    U = Y + 9.0 * (1 - ops.poisson_node_interior(Y.shape).numpy()) * rng.standard_normal(Y.shape)
    R = ops.cavity_node_residual(_cavity_node_spec(n, lid=1.0), [torch.tensor(U), torch.tensor(z), torch.tensor(z)])
    for r in R:
        assert float(r[:, 1:-1].abs().max()) < 1e-13
    # next to the left wall u drops to 0: u_x = (y - 0) / 2h, u_xx = (y - 2 y + 0) / h^2
    h, yi = 1.0 / n, y[1:-1]
    np.testing.assert_allclose(R[1][:, 0].numpy(), yi * yi / (2 * h) + (1 / 100.0) * yi / h ** 2,
                               rtol=1e-12)


def test_cavity_node_pressure_neumann_wall():
    """p = s x at rest: a zero normal derivative at the wall makes the wall
    pressure equal its neighbour's, so the node next to the wall sees half the
    slope in the momentum equation and a one-sided stabilisation term in
    continuity; elsewhere p_x = s exactly and the stabilisation vanishes."""
    n, s, tau = 8, 3.0, 0.5
    x = np.arange(n + 1) / n
    P = np.tile(s * x[None, :], (n + 1, 1))
    z = np.zeros_like(P)
    R = ops.cavity_node_residual(_cavity_node_spec(n, tau=tau), [torch.tensor(z), torch.tensor(z), torch.tensor(P)])
    cont, mu, mv = (r.numpy() for r in R)
    np.testing.assert_allclose(mu[:, 1:-1], s, rtol=1e-13)
    np.testing.assert_allclose(mu[:, 0], s / 2, rtol=1e-13)
    np.testing.assert_allclose(mu[:, -1], s / 2, rtol=1e-13)
    np.testing.assert_allclose(cont[:, 1:-1], 0.0, atol=1e-12)
    np.testing.assert_allclose(cont[:, 0], -tau * s, rtol=1e-12)
    np.testing.assert_allclose(cont[:, -1], tau * s, rtol=1e-12)
    assert float(np.abs(mv).max()) == 0.0


def test_cavity_node_wall_values_do_not_matter():
    """Every wall node's value is replaced (velocity imposed, pressure copied):
    the loss does not depend on the fine field there and its gradient is zero."""
    spec = _cavity_node_spec(8, re=400.0, lid=1.0)
    spec.forcing = {}
    rng = np.random.default_rng(11)
    f = [rng.standard_normal((9, 9)) for _ in range(3)]
    mask = ops.poisson_node_interior((9, 9)).numpy()
    g = [x * mask + 5.0 * (1 - mask) * rng.standard_normal((9, 9)) for x in f]
    assert ops.loss_value(spec, [f])["pde"] == ops.loss_value(spec, [g])["pde"]
    _, gr = ops.loss_and_grad(spec, [f])
    for c in range(3):
        assert np.all(gr[0][c][mask == 0] == 0.0)
        assert np.linalg.norm(gr[0][c]) > 0


def test_cavity_node_pressure_gauge_invariance():
    spec = _cavity_node_spec(8, re=400.0, lid=1.0)
    rng = np.random.default_rng(3)
    f = [rng.standard_normal((9, 9)) for _ in range(3)]
    a = ops.loss_value(spec, [f])["pde"]
    b = ops.loss_value(spec, [[f[0], f[1], f[2] + 3.25]])["pde"]
    assert abs(a - b) <= 1e-13 * a


def test_cavity_node_level_shapes():
    assert ops.level_shapes("cavity", (64, 64), 5, "node") == [[(n, n)] * 3 for n in (65, 33, 17, 9, 5)]


# ------------------------------------------------------- node-based Poisson
def _node_grid(n, d):
    x = np.arange(n + 1) / n
    return np.meshgrid(*([x] * d), indexing="ij")


@pytest.mark.parametrize("d", [1, 2, 3])
def test_node_poisson_exact_for_product_of_quadratics(d):
    """u = prod x_a (1 - x_a) vanishes on the boundary, and the 3-point second
    difference of x (1 - x) is exactly -2, so f = -2 sum_a prod_{b != a}
    x_b (1 - x_b) makes every term of the node-based loss zero."""
    n = 8
    X = _node_grid(n, d)
    q = [x * (1 - x) for x in X]
    u = np.prod(q, axis=0)
    f = np.zeros_like(u)
    for a in range(d):
        f += -2.0 * np.prod([q[b] for b in range(d) if b != a], axis=0) if d > 1 else -2.0
    spec = ops.Spec("poisson", (n,) * d, (1.0,) * d, 1, weights={"pde": 1.0, "bc": 1.0},
                    centering="node", forcing={0: f})
    terms = ops.loss_value(spec, [[u]])
    assert terms["pde"] < 1e-26 and terms["bc"] < 1e-30, terms


@pytest.mark.parametrize("d", [1, 2, 3])
def test_node_boundary_values_are_imposed(d):
    """The boundary nodes carry the Dirichlet value itself: the loss does not
    depend on the fine field there, and its gradient there is zero."""
    n = 8
    rng = np.random.default_rng(d)
    spec = ops.Spec("poisson", (n,) * d, (1.0,) * d, 1, weights={"pde": 1.0, "bc": 1.0},
                    centering="node", forcing={0: rng.standard_normal((n + 1,) * d)})
    u = rng.standard_normal((n + 1,) * d)
    mask = ops.poisson_node_interior(u.shape).numpy()
    t1 = ops.loss_value(spec, [[u]])
    t2 = ops.loss_value(spec, [[u * mask + 7.0 * (1 - mask)]])
    assert t1 == t2
    _, g = ops.loss_and_grad(spec, [[u]])
    assert np.all(g[0][0][mask == 0] == 0.0)
    assert np.linalg.norm(g[0][0]) > 0


def test_node_level_shapes():
    assert ops.level_shapes("poisson", (32, 16), 3, "node") == [[(33, 17)], [(17, 9)], [(9, 5)]]


def test_node_lbfgs_converges_fast_in_1d():
    """Section 3.1: in 1-D, L-BFGS reaches machine precision in about 50
    iterations with three or more levels (node-based)."""
    from oracle import lbfgs as ol
    n = 32
    x = np.arange(n + 1) / n
    v = 5.0 * (1.0 - x) * x
    u_ref = (v ** 5 / (1.0 + v ** 5)) ** 0.2
    f = np.zeros(n + 1)
    f[1:-1] = (u_ref[2:] - 2 * u_ref[1:-1] + u_ref[:-2]) * n * n
    spec = ops.Spec("poisson", (n,), (1.0,), 3, weights={"pde": 1.0, "bc": 1.0},
                    centering="node", forcing={0: f})
    shapes = ops.level_shapes("poisson", (n,), 3, "node")
    sizes = [s[0][0] for s in shapes]

    def split(xv):
        out, o = [], 0
        for m in sizes:
            out.append([xv[o:o + m]])
            o += m
        return out

    def fg(xv):
        t, g = ops.loss_and_grad(spec, split(xv))
        return sum(t.values()), np.concatenate([gg[0] for gg in g])

    it = ol.LBFGS(fg, np.zeros(sum(sizes)), m=50)
    for k in range(80):
        if it.step().status == 2:
            break
    fine = ops.fine_fields(spec, [[torch.as_tensor(a[0])] for a in split(it.x)])[0].numpy()
    fine = fine * ops.poisson_node_interior(fine.shape).numpy()  # boundary values imposed
    assert np.max(np.abs(fine - u_ref)) < 1e-12, (k, np.max(np.abs(fine - u_ref)))


# ---------------------------------------------------- node-based channel flow
_NS_NODE = {"re": 50.0, "diam": 0.4, "lam": 2.0, "chi_shift": 5.0, "tau_coef": 0.5}


def _channel_node_spec(dims, lengths, chi, u_ref=0.8, forcing=None):
    return ops.Spec("ns3d_fixed", dims, lengths, 1, params=dict(_NS_NODE, u_ref=u_ref),
                    weights={"pde": 1.0}, chi=chi, centering="node", forcing=forcing or {})


def _channel_grid(dims, lengths):
    axes = [np.arange(n + 1) * (L / n) for n, L in zip(dims, lengths)]
    return np.meshgrid(*axes, indexing="ij")   # Z, Y, X


def _scramble_boundary(f, seed):
    """Replace every boundary node's value by noise (the operator must not read it)."""
    inside = ops.poisson_node_interior(f.shape).numpy()
    rng = np.random.default_rng(seed)
    return f * inside + 7.0 * (1 - inside) * rng.standard_normal(f.shape)


def _channel(spec, u, v, w, p, seed=None):
    fs = [u, v, w, p]
    if seed is not None:
        fs = [_scramble_boundary(f, seed + k) for k, f in enumerate(fs)]
    return [r.numpy() for r in ops.channel_node_residual(spec, [torch.tensor(f) for f in fs])]


def test_channel_node_exact_for_products_of_quadratics():
    """Fields that are quadratic along each axis separately, where central
    first and second differences are exact: away from the boundary (nodes
    whose stars touch no boundary node) the node residuals are the continuous
    penalised Navier-Stokes operators with the pressure stabilisation
    tau h_a d2p/da2, body fraction included."""
    dims, lengths = (6, 6, 10), (1.0, 1.2, 2.0)
    Z, Y, X = _channel_grid(dims, lengths)
    rng = np.random.default_rng(17)

    def quad(s):
        a, b, c = rng.uniform(-1, 1, 3)
        return a + b * s + c * s * s, b + 2 * c * s, 2 * c * np.ones_like(s)

    F = []   # (value, first derivatives along z, y, x, second derivatives along z, y, x)
    for _ in range(4):
        (qz, dz, zz), (qy, dy, yy), (qx, dx, xx) = quad(Z), quad(Y), quad(X)
        F.append((qz * qy * qx, (dz * qy * qx, qz * dy * qx, qz * qy * dx),
                  (zz * qy * qx, qz * yy * qx, qz * qy * xx)))
    chi = rng.uniform(0, 1, size=Z.shape)
    h = tuple(L / n for L, n in zip(lengths, dims))
    nu, lam, tau = 0.4 / 50.0, 2.0, 0.5
    vel, P = F[:3], F[3]
    axis_of = [2, 1, 0]   # velocity component c points along axis 2 - c
    R = _channel(_channel_node_spec(dims, lengths, chi), *(f[0] for f in vel), P[0])
    for r in R:
        assert r.shape == tuple(d - 1 for d in dims)
    deep = (slice(2, -2),) * 3      # on the node grid
    rdeep = (slice(1, -1),) * 3     # on the interior-node arrays
    cont = sum(vel[c][1][axis_of[c]] for c in range(3)) - sum(tau * h[a] * P[2][a] for a in range(3))
    np.testing.assert_allclose(R[0][rdeep], cont[deep], rtol=1e-11, atol=1e-11)
    for c in range(3):
        body = (sum(vel[k][0] * vel[c][1][axis_of[k]] for k in range(3)) + P[1][axis_of[c]]
                - nu * sum(vel[c][2]))
        want = (1 - chi) * body + lam * chi * vel[c][0]
        np.testing.assert_allclose(R[1 + c][rdeep], want[deep], rtol=1e-11, atol=1e-11)


def test_channel_node_uniform_flow_is_exact():
    """The free stream u = (u_ref, 0, 0), p = 0 without a body satisfies every
    boundary condition: all residuals vanish, whatever the boundary nodes hold."""
    dims, lengths = (4, 6, 8), (1.0, 1.0, 2.0)
    shape = tuple(d + 1 for d in dims)
    z = np.zeros(shape)
    R = _channel(_channel_node_spec(dims, lengths, z), np.full(shape, 0.8), z, z, z, seed=3)
    for r in R:
        assert float(np.abs(r).max()) == 0.0


def test_channel_node_inlet_and_outlet():
    """u = u_ref + a x, p = s (x - L) without a body.  The inlet imposes
    u = u_ref (on the line) and copies p from the first interior node; the
    outlet imposes p = 0 (on the line) and copies the velocity.  Next to the
    inlet the pressure sees half the slope and a one-sided second difference;
    next to the outlet the velocity does; elsewhere the line is exact."""
    dims, lengths = (4, 4, 8), (1.0, 1.0, 2.0)
    Z, Y, X = _channel_grid(dims, lengths)
    a, s, u_ref = 0.3, -1.5, 0.8
    h, nx = lengths[2] / dims[2], dims[2]
    nu, tau = 0.4 / 50.0, 0.5
    spec = _channel_node_spec(dims, lengths, np.zeros(X.shape), u_ref=u_ref)
    z = np.zeros(X.shape)
    cont, mu, mv, mw = _channel(spec, u_ref + a * X, z, z, s * (X - lengths[2]), seed=9)
    xi = np.arange(1, nx) * h
    ux = np.full(nx - 1, a)
    uxx = np.zeros(nx - 1)
    ux[-1], uxx[-1] = a / 2, -a / h
    px = np.full(nx - 1, s)
    pxx = np.zeros(nx - 1)
    px[0], pxx[0] = s / 2, s / h
    # the outlet node copies u(N-1), so the node next to it sees u = u_ref + a x there
    ui = u_ref + a * xi
    want_cont = ux - tau * h * pxx
    want_mu = ui * ux + px - nu * uxx
    for zi in range(dims[0] - 1):
        for yi in range(dims[1] - 1):
            np.testing.assert_allclose(cont[zi, yi], want_cont, rtol=1e-12, atol=1e-13)
            np.testing.assert_allclose(mu[zi, yi], want_mu, rtol=1e-12, atol=1e-13)
    assert float(np.abs(mv).max()) == 0.0 and float(np.abs(mw).max()) == 0.0


@pytest.mark.parametrize("wall_axis", [0, 1])
def test_channel_node_free_slip_walls(wall_axis):
    """Across the walls of axis 0 (z) or 1 (y): the normal component n = b q,
    q = s (L - s), vanishes on the wall and is quadratic, so it is exact; the
    tangential u = u_ref + c s is copied to the wall node (zero normal
    derivative), which halves its slope and gives a one-sided second difference
    next to the wall.  Checked away from the inlet and outlet."""
    dims, lengths = (6, 6, 8), (1.0, 1.0, 2.0)
    G = _channel_grid(dims, lengths)
    S = G[wall_axis]
    Ls, n = lengths[wall_axis], dims[wall_axis]
    h = Ls / n
    b, c, u_ref = 0.7, 0.4, 0.8
    nu = 0.4 / 50.0
    z = np.zeros(S.shape)
    normal = b * S * (Ls - S)
    u = u_ref + c * S
    v, w = (normal, z) if wall_axis == 1 else (z, normal)
    spec = _channel_node_spec(dims, lengths, z, u_ref=u_ref)
    cont, mu, mv, mw = _channel(spec, u, v, w, z, seed=21)
    si = np.arange(1, n) * h
    us = np.full(n - 1, c)
    uss = np.zeros(n - 1)
    us[0] = us[-1] = c / 2
    uss[0], uss[-1] = c / h, -c / h
    nv = b * si * (Ls - si)
    ns = b * (Ls - 2 * si)
    want = {"cont": ns, "mu": nv * us - nu * uss, "mn": nv * ns + 2 * nu * b}
    mn, mt = (mv, mw) if wall_axis == 1 else (mw, mv)
    xs = slice(1, -1)   # away from the inlet and outlet nodes' neighbours
    for name, arr in (("cont", cont), ("mu", mu), ("mn", mn)):
        arr = np.moveaxis(arr, wall_axis, 0)[:, :, xs]
        np.testing.assert_allclose(arr, np.broadcast_to(want[name][:, None, None], arr.shape),
                                   rtol=1e-12, atol=1e-13, err_msg=name)
    assert float(np.abs(mt).max()) == 0.0


def test_channel_node_boundary_values_do_not_matter():
    """Every boundary node's value is replaced (imposed or copied): the loss
    does not depend on the fine field there and its gradient is zero."""
    dims = (4, 4, 8)
    shape = tuple(d + 1 for d in dims)
    spec = ops.Spec("ns3d", dims, (1.0, 1.0, 2.0), 1, params=dict(_NS_NODE, u_ref=1.0),
                    weights={"pde": 1.0}, centering="node")
    rng = np.random.default_rng(12)
    f = [rng.standard_normal(shape) for _ in range(5)]
    g = [_scramble_boundary(x, 40 + k) for k, x in enumerate(f)]
    assert ops.loss_value(spec, [f])["pde"] == ops.loss_value(spec, [g])["pde"]
    _, gr = ops.loss_and_grad(spec, [f])
    mask = ops.poisson_node_interior(shape).numpy()
    for k in range(5):
        assert np.all(gr[0][k][mask == 0] == 0.0)
        assert np.linalg.norm(gr[0][k]) > 0


def test_channel_node_level_shapes():
    assert ops.level_shapes("ns3d", (64, 64, 128), 3, "node") == \
        [[(65, 65, 129)] * 5, [(33, 33, 65)] * 5, [(17, 17, 33)] * 5]
