"""Discrete residuals and loss terms of the ODIL problems (paper Sections 2.1, 3).

Every problem is a loss over discrete fields on a uniform cell-centred grid:
a weighted sum of squared residuals of the discretised PDE (integrals are
sums times the cell measure), data terms (means over the measurement
points), and regularisation / initial / boundary terms (Section 2.1).  The
loss is evaluated on the fine field u = M_L(u_1..u_L); the gradient with
respect to every level follows by automatic differentiation, exactly as in
the paper.

Where the paper leaves a discretisation detail open, the reading below is
the one the whole project uses (every reading is listed in the design notes):

  poisson  d-dimensional Laplacian, Dirichlet u = 0 through quadratic
           extrapolation from the two nearest cell centres and the face
           value (Section 3.1); forcing f defined as the discrete Laplacian of
           the reference solution, so that it is the exact discrete solution.
  burgers  u_t + (u^2/2)_x = 0 on a space-time grid, implicit first-order
           upwind flux (Murman-Roe form) on the inner points, data mean,
           gradient-squared smoothing in x and t (Section 3.2).
  heat     u_t = (k(x) u_x)_x with k = softplus(q), implicit scheme of
           Section 3.4 with the face conductivity the mean of the adjacent
           cells, quadratic extrapolation to impose u = 0 on the walls, an
           initial-condition term and a data mean.
  ns3d     steady incompressible Navier-Stokes with Brinkman penalisation
           (Section 3.5): central differences on a collocated grid with a
           compact pressure-stabilised continuity equation, body fraction
           chi = sigmoid(chihat - shift), inlet/outlet/free-slip ghost rules.
  cavity   steady 2-D Navier-Stokes in the lid-driven cavity (Section 3.3),
           same discretisation as ns3d, no-slip walls, unit lid velocity;
           cell-based, or node-based with the wall velocity imposed on the
           wall nodes.

Optional per-equation forcing arrays (fine grid) are subtracted from the
residuals; they let a test manufacture a state whose residual is zero.
"""
import math

import torch

from . import multigrid

DT = torch.float64

# field names and the grid axes each field spans, per problem
FIELDS = {
    "poisson": ["u"],
    "burgers": ["u"],
    "heat": ["u", "q"],
    "ns3d": ["u", "v", "w", "p", "chihat"],
    "ns3d_fixed": ["u", "v", "w", "p"],
    "cavity": ["u", "v", "p"],
}

TERMS = ("pde", "data", "reg", "ic", "bc")


def field_axes(op, field, ndim):
    """Axes of the fine grid that a field spans (q of the heat problem is 1-D in x)."""
    if op == "heat" and field == "q":
        return (0,)
    return tuple(range(ndim))


def field_shape(op, field, dims):
    if op == "heat" and field == "q":
        return (dims[1],)
    return tuple(dims)


def level_shapes(op, dims, n_levels, centering="cell"):
    """Shape of every (level, field) array: list over levels of list over fields.

    dims are cells per axis; node-based fields hold one more value per axis
    (the nodes, boundary nodes included)."""
    extra = 1 if centering == "node" else 0
    out = []
    for lvl in range(n_levels):
        row = []
        for f in FIELDS[op]:
            s = field_shape(op, f, dims)
            row.append(tuple(n // 2 ** lvl + extra for n in s))
        out.append(row)
    return out


class Spec:
    """Plain description of one problem instance for the oracle.

    op         one of FIELDS
    dims       fine-grid cells per axis, slowest axis first
    lengths    domain extent per axis (same order)
    n_levels   number of multigrid levels L
    params     dict of physical constants (re, diam, lam, chi_shift, tau_coef)
    weights    dict of term weights (pde, data, reg, ic, bc)
    meas       list of (field_index, term, flat_cell_index array, values, weight)
               weight multiplies every squared misfit of that list
    forcing    dict eq_index -> fine-grid array subtracted from residual eq
    chi        fixed body fraction (ns3d_fixed only)
    """

    def __init__(self, op, dims, lengths, n_levels, params=None, weights=None,
                 meas=None, forcing=None, chi=None, centering="cell"):
        self.op = op
        self.dims = tuple(int(d) for d in dims)
        self.lengths = tuple(float(x) for x in lengths)
        self.n_levels = int(n_levels)
        self.params = dict(params or {})
        self.weights = {t: 0.0 for t in TERMS}
        self.weights.update(weights or {})
        self.meas = list(meas or [])
        self.forcing = dict(forcing or {})
        self.chi = chi
        self.centering = centering

    @property
    def ndim(self):
        return len(self.dims)

    @property
    def h(self):
        return tuple(L / n for L, n in zip(self.lengths, self.dims))

    @property
    def cell_measure(self):
        return math.prod(self.h)

    @property
    def fields(self):
        return FIELDS[self.op]


# ------------------------------------------------------------- ghost padding
def _pad(x, axis, lo, hi):
    """Append ghost slabs `lo` and `hi` (callables of x moved to axis 0)."""
    y = torch.movedim(x, axis, 0)
    g0 = lo(y).unsqueeze(0)
    g1 = hi(y).unsqueeze(0)
    return torch.movedim(torch.cat([g0, y, g1], 0), 0, axis)


def _dirichlet(b):
    """Ghost value making the face mean equal to b (linear): 2b - interior."""
    return (lambda y: 2.0 * b - y[0]), (lambda y: 2.0 * b - y[-1])


def _dirichlet_lo(b):
    return lambda y: 2.0 * b - y[0]


def _dirichlet_hi(b):
    return lambda y: 2.0 * b - y[-1]


def _neumann_lo(y):
    return y[0]


def _neumann_hi(y):
    return y[-1]


def _quad_zero_lo(y):
    # quadratic through (face, 0), (x_0, y0), (x_1, y1) evaluated one cell
    # outside: Lagrange weights 8/3, -2, 1/3 at face, first, second centre
    return -2.0 * y[0] + y[1] / 3.0


def _quad_zero_hi(y):
    return -2.0 * y[-1] + y[-2] / 3.0


def _shift(xp, axis, s):
    """Slice of a padded array (1 ghost per side) at offset s in {-1,0,1}."""
    n = xp.shape[axis] - 2
    return torch.narrow(xp, axis, 1 + s, n)


# ------------------------------------------------------------------ residuals
def poisson_node_residual(spec, u):
    """Node-based Poisson (Section 3.1): the finite-difference Laplacian minus
    the forcing at the interior nodes.  The zero Dirichlet condition is imposed
    on the boundary nodes directly: the fine field's boundary values are
    replaced by zero before the stencil is applied, so they carry no unknown
    and the boundary integral of u^2 in the loss vanishes."""
    u = u * poisson_node_interior(u.shape)
    inner = tuple(slice(1, -1) for _ in range(u.dim()))
    f = spec.forcing.get(0)
    R = torch.zeros_like(u[inner]) if f is None else -torch.as_tensor(f, dtype=DT)[inner]
    for a, h in enumerate(spec.h):
        lo = tuple(slice(0, -2) if b == a else slice(1, -1) for b in range(u.dim()))
        hi = tuple(slice(2, None) if b == a else slice(1, -1) for b in range(u.dim()))
        R = R + (u[hi] - 2.0 * u[inner] + u[lo]) / h ** 2
    return [R]


def poisson_node_interior(shape):
    """1 at the interior nodes, 0 at the boundary nodes (index 0 or N on some axis)."""
    m = torch.ones(shape, dtype=DT)
    for a in range(len(shape)):
        idx = [slice(None)] * len(shape)
        idx[a] = 0
        m[tuple(idx)] = 0.0
        idx[a] = -1
        m[tuple(idx)] = 0.0
    return m


def poisson_residual(spec, u):
    """Laplacian minus forcing at every cell (Section 3.1, cell-based)."""
    f = spec.forcing.get(0)
    R = torch.zeros_like(u) if f is None else -torch.as_tensor(f, dtype=DT)
    for a, h in enumerate(spec.h):
        up = _pad(u, a, _quad_zero_lo, _quad_zero_hi)
        R = R + (_shift(up, a, 1) - 2.0 * u + _shift(up, a, -1)) / h ** 2
    return [R]


def _upwind_flux(a, b):
    """First-order upwind flux of u^2/2 between states a (left) and b (right).

    Murman-Roe form: mean of the two physical fluxes minus half the absolute
    face speed times the jump; it takes the left flux when the face speed
    (a+b)/2 is positive and the right one when it is negative.
    """
    return 0.25 * (a * a + b * b) - 0.5 * torch.abs(0.5 * (a + b)) * (b - a)


def burgers_residual(spec, u):
    """Implicit upwind finite-volume residual on the inner points (Section 3.2).

    Rows are time levels (row 0 is the initial state), columns are cells.
    """
    dt, dx = spec.h
    un = u[1:, 1:-1]
    R = (un - u[:-1, 1:-1]) / dt + (_upwind_flux(un, u[1:, 2:])
                                    - _upwind_flux(u[1:, :-2], un)) / dx
    f = spec.forcing.get(0)
    if f is not None:
        R = R - torch.as_tensor(f, dtype=DT)[1:, 1:-1]
    return [R]


def burgers_smoothing(spec, u):
    """Gradient-squared regularisation terms on all inner faces (Section 3.2)."""
    dt, dx = spec.h
    gx = (u[:, 1:] - u[:, :-1]) / dx
    gt = (u[1:, :] - u[:-1, :]) / dt
    return gx, gt


def softplus(q):
    """log(1 + e^q) in a form that neither overflows nor loses digits."""
    pos = q + torch.log1p(torch.exp(-torch.clamp(q, min=0.0)))
    neg = torch.log1p(torch.exp(torch.clamp(q, max=0.0)))
    return torch.where(q > 0, pos, neg)


def heat_residual(spec, u, q):
    """Implicit heat-equation residual with conductivity k(x) = softplus(q).

    Section 3.4 scheme, with the face conductivity the mean of the two
    adjacent cell conductivities.  Inner points only: rows n >= 1, columns
    1..N-2.
    """
    dt, dx = spec.h
    k = softplus(q)
    kp = 0.5 * (k[1:-1] + k[2:])
    km = 0.5 * (k[1:-1] + k[:-2])
    un = u[1:, 1:-1]
    R = (un - u[:-1, 1:-1]) / dt - (kp * (u[1:, 2:] - un) - km * (un - u[1:, :-2])) / dx ** 2
    f = spec.forcing.get(0)
    if f is not None:
        R = R - torch.as_tensor(f, dtype=DT)[1:, 1:-1]
    return [R]


def heat_boundary(spec, u):
    """Wall value u(face) from quadratic extrapolation of the 3 nearest cells.

    Rows n >= 1 (row 0 is fixed by the initial-condition term).
    """
    left = (15.0 * u[1:, 0] - 10.0 * u[1:, 1] + 3.0 * u[1:, 2]) / 8.0
    right = (15.0 * u[1:, -1] - 10.0 * u[1:, -2] + 3.0 * u[1:, -3]) / 8.0
    return left, right


def _ns_ghost_rules_3d():
    """Ghost rules for (u, v, w, p) on axes (z, y, x) of the channel (Section 3.5).

    x: inlet u = (1, 0, 0) at x = 0 (Dirichlet), p Neumann; outlet p = 0 at
    the far end (Dirichlet), velocity Neumann.  y and z: free-slip walls, the
    normal velocity component is zero (Dirichlet), tangential components and p
    are Neumann.
    """
    D, N = _dirichlet_lo, _dirichlet_hi
    rules = {}
    # axis 2 = x
    rules[(0, 2)] = (D(1.0), _neumann_hi)      # u
    rules[(1, 2)] = (D(0.0), _neumann_hi)      # v
    rules[(2, 2)] = (D(0.0), _neumann_hi)      # w
    rules[(3, 2)] = (_neumann_lo, N(0.0))      # p
    # axis 1 = y (normal component v)
    rules[(0, 1)] = (_neumann_lo, _neumann_hi)
    rules[(1, 1)] = (D(0.0), N(0.0))
    rules[(2, 1)] = (_neumann_lo, _neumann_hi)
    rules[(3, 1)] = (_neumann_lo, _neumann_hi)
    # axis 0 = z (normal component w)
    rules[(0, 0)] = (_neumann_lo, _neumann_hi)
    rules[(1, 0)] = (_neumann_lo, _neumann_hi)
    rules[(2, 0)] = (D(0.0), N(0.0))
    rules[(3, 0)] = (_neumann_lo, _neumann_hi)
    return rules


def _cavity_ghost_rules():
    """Ghost rules for (u, v, p) on axes (y, x): no-slip walls, lid u = 1 at y = 1."""
    D, N = _dirichlet_lo, _dirichlet_hi
    rules = {}
    rules[(0, 1)] = (D(0.0), N(0.0))           # u on x walls
    rules[(1, 1)] = (D(0.0), N(0.0))           # v on x walls
    rules[(2, 1)] = (_neumann_lo, _neumann_hi)  # p
    rules[(0, 0)] = (D(0.0), N(1.0))           # u: bottom wall, moving lid
    rules[(1, 0)] = (D(0.0), N(0.0))
    rules[(2, 0)] = (_neumann_lo, _neumann_hi)
    return rules


def _navier_stokes(spec, vel, p, chi, rules, nu, lam, tau_coef):
    """Momentum and continuity residuals of the penalised steady NS equations.

    vel[c] is the velocity component along axis (ndim-1-c) (u along the last,
    fastest axis).  Returns [continuity, momentum_0, momentum_1, ...].
    """
    nd = spec.ndim
    h = spec.h
    comp_axis = [nd - 1 - c for c in range(nd)]
    padded = {}
    for c in range(nd):
        for a in range(nd):
            lo, hi = rules[(c, a)]
            padded[(c, a)] = _pad(vel[c], a, lo, hi)
    for a in range(nd):
        lo, hi = rules[(nd, a)]
        padded[(nd, a)] = _pad(p, a, lo, hi)

    def d1(fi, a):   # central first difference along axis a
        xp = padded[(fi, a)]
        return (_shift(xp, a, 1) - _shift(xp, a, -1)) / (2.0 * h[a])

    def lap(fi, center):
        out = 0.0
        for a in range(nd):
            xp = padded[(fi, a)]
            out = out + (_shift(xp, a, 1) - 2.0 * center + _shift(xp, a, -1)) / h[a] ** 2
        return out

    cont = 0.0
    for c in range(nd):
        cont = cont + d1(c, comp_axis[c])
    stab = 0.0
    for a in range(nd):
        xp = padded[(nd, a)]
        stab = stab + tau_coef * h[a] * (_shift(xp, a, 1) - 2.0 * p + _shift(xp, a, -1)) / h[a] ** 2
    res = [cont - stab]
    for c in range(nd):
        conv = 0.0
        for k in range(nd):
            conv = conv + vel[k] * d1(c, comp_axis[k])
        body = conv + d1(nd, comp_axis[c]) - nu * lap(c, vel[c])
        if chi is None:
            res.append(body)
        else:
            res.append((1.0 - chi) * body + lam * chi * vel[c])
    for e in range(len(res)):
        f = spec.forcing.get(e)
        if f is not None:
            res[e] = res[e] - torch.as_tensor(f, dtype=DT)
    return res


def ns3d_chi(spec, chihat):
    """Body fraction chi = 1 / (1 + exp(-(chihat - shift)))  (Section 3.5)."""
    return torch.sigmoid(chihat - spec.params.get("chi_shift", 5.0))


def ns3d_residual(spec, fields):
    u, v, w, p = fields[:4]
    if spec.op == "ns3d":
        chi = ns3d_chi(spec, fields[4])
    else:
        chi = torch.as_tensor(spec.chi, dtype=DT)
    P = spec.params
    nu = P.get("diam", 0.4) / P["re"]
    return _navier_stokes(spec, [u, v, w], p, chi, _ns_ghost_rules_3d(), nu,
                          P.get("lam", 1.0), P.get("tau_coef", 0.5))


def cavity_residual(spec, fields):
    u, v, p = fields
    P = spec.params
    return _navier_stokes(spec, [u, v], p, None, _cavity_ghost_rules(), 1.0 / P["re"],
                          0.0, P.get("tau_coef", 0.5))


def cavity_node_residual(spec, fields):
    """Lid-driven cavity on node-based values (Sections 2.2, 3.3).

    Nodes x_i = i h, i = 0..N on both axes.  The no-slip condition is imposed
    on the wall nodes directly: their velocity is zero, except u = u_ref on the
    lid's nodes (y = 1, the two corners excluded), whatever the fine field
    holds there.  The wall pressure is that of the interior node next to it
    (zero normal derivative).  Continuity and momentum hold at the interior
    nodes, with central differences and the stabilised continuity equation of
    the cell-based form.  Returns [continuity, momentum u, momentum v] on the
    interior nodes."""
    u, v, p = fields
    lid = spec.params.get("u_ref", 1.0)
    inside = poisson_node_interior(u.shape)
    top = torch.zeros_like(u)
    top[-1, 1:-1] = lid  # axis 0 = y: the last row is the lid
    u = u * inside + top
    v = v * inside
    p = p.clone()
    p[0, :] = p[1, :]
    p[-1, :] = p[-2, :]
    p[:, 0] = p[:, 1]
    p[:, -1] = p[:, -2]
    hy, hx = spec.h
    P = spec.params
    nu = 1.0 / P["re"]
    tau = P.get("tau_coef", 0.5)
    inner = (slice(1, -1), slice(1, -1))

    def dx(f):
        return (f[1:-1, 2:] - f[1:-1, :-2]) / (2.0 * hx)

    def dy(f):
        return (f[2:, 1:-1] - f[:-2, 1:-1]) / (2.0 * hy)

    def lap_x(f):
        return (f[1:-1, 2:] - 2.0 * f[inner] + f[1:-1, :-2]) / hx ** 2

    def lap_y(f):
        return (f[2:, 1:-1] - 2.0 * f[inner] + f[:-2, 1:-1]) / hy ** 2

    uc, vc = u[inner], v[inner]
    cont = dx(u) + dy(v) - (tau * hx * lap_x(p) + tau * hy * lap_y(p))
    mom_u = uc * dx(u) + vc * dy(u) + dx(p) - nu * (lap_x(u) + lap_y(u))
    mom_v = uc * dx(v) + vc * dy(v) + dy(p) - nu * (lap_x(v) + lap_y(v))
    res = [cont, mom_u, mom_v]
    for e in range(3):
        f = spec.forcing.get(e)
        if f is not None:
            res[e] = res[e] - torch.as_tensor(f, dtype=DT)[inner]
    return res


def channel_node_residual(spec, fields):
    """Channel flow past a body on node-based values (Sections 2.2, 3.5).

    Nodes x_i = i h on each axis (z, y, x).  Boundary nodes carry no equation;
    the boundary conditions are imposed on their values, whatever the fine
    field holds there:
      inlet (x = 0)      u = (u_ref, 0, 0); p of the interior node next to it,
      outlet (x = L)     p = 0; the velocity of the interior node next to it,
      walls (y, z ends)  free slip: the normal velocity component is zero, the
                         other components and p are those of the interior node
                         next to the wall.
    Nodes on an edge or a corner of the box lie in no interior node's 7-point
    star, so the order of these substitutions does not matter.  Continuity
    (with the pressure stabilisation) and the penalised momentum equations
    hold at the interior nodes with central differences, as in the cell-based
    form.  Returns [continuity, momentum u, momentum v, momentum w] on the
    interior nodes."""
    u, v, w, p = (x.clone() for x in fields[:4])
    P = spec.params
    u_ref = P.get("u_ref", 1.0)
    # inlet and outlet (axis 2)
    u[:, :, 0] = u_ref
    v[:, :, 0] = 0.0
    w[:, :, 0] = 0.0
    p[:, :, 0] = p[:, :, 1]
    for f in (u, v, w):
        f[:, :, -1] = f[:, :, -2]
    p[:, :, -1] = 0.0
    # free-slip walls: y ends (normal component v), z ends (normal component w)
    for f in (u, w, p):
        f[:, 0, :] = f[:, 1, :]
        f[:, -1, :] = f[:, -2, :]
    v[:, 0, :] = 0.0
    v[:, -1, :] = 0.0
    for f in (u, v, p):
        f[0, :, :] = f[1, :, :]
        f[-1, :, :] = f[-2, :, :]
    w[0, :, :] = 0.0
    w[-1, :, :] = 0.0

    h = spec.h
    inner = (slice(1, -1),) * 3

    def nb(f, a, s):   # values of the neighbours at offset s along axis a
        idx = list(inner)
        idx[a] = slice(1 + s, f.shape[a] - 1 + s)
        return f[tuple(idx)]

    def d1(f, a):
        return (nb(f, a, 1) - nb(f, a, -1)) / (2.0 * h[a])

    def d2(f, a):
        return (nb(f, a, 1) - 2.0 * f[inner] + nb(f, a, -1)) / h[a] ** 2

    vel = [u, v, w]           # component c points along axis 2 - c
    axis_of = [2, 1, 0]
    if spec.op == "ns3d":
        chi = ns3d_chi(spec, fields[4])[inner]
    else:
        chi = torch.as_tensor(spec.chi, dtype=DT)[inner]
    nu = P.get("diam", 0.4) / P["re"]
    lam = P.get("lam", 1.0)
    tau = P.get("tau_coef", 0.5)
    cont = sum(d1(vel[c], axis_of[c]) for c in range(3))
    cont = cont - sum(tau * h[a] * d2(p, a) for a in range(3))
    res = [cont]
    for c in range(3):
        conv = sum(vel[k][inner] * d1(vel[c], axis_of[k]) for k in range(3))
        lap = sum(d2(vel[c], a) for a in range(3))
        body = conv + d1(p, axis_of[c]) - nu * lap
        res.append((1.0 - chi) * body + lam * chi * vel[c][inner])
    for e in range(4):
        f = spec.forcing.get(e)
        if f is not None:
            res[e] = res[e] - torch.as_tensor(f, dtype=DT)[inner]
    return res


def residuals(spec, fine):
    """PDE residual arrays of the problem for the list of fine fields."""
    op = spec.op
    if op == "poisson" and spec.centering == "node":
        return poisson_node_residual(spec, fine[0])
    if op == "cavity" and spec.centering == "node":
        return cavity_node_residual(spec, fine)
    if op in ("ns3d", "ns3d_fixed") and spec.centering == "node":
        return channel_node_residual(spec, fine)
    if op == "poisson":
        return poisson_residual(spec, fine[0])
    if op == "burgers":
        return burgers_residual(spec, fine[0])
    if op == "heat":
        return heat_residual(spec, fine[0], fine[1])
    if op in ("ns3d", "ns3d_fixed"):
        return ns3d_residual(spec, fine)
    if op == "cavity":
        return cavity_residual(spec, fine)
    raise ValueError(op)


# ------------------------------------------------------------------- the loss
def loss_terms(spec, fine):
    """Loss terms (pde, data, reg, ic, bc) as 0-d FP64 tensors."""
    W = spec.weights
    V = spec.cell_measure
    terms = {t: torch.zeros((), dtype=DT) for t in TERMS}
    R = residuals(spec, fine)
    terms["pde"] = W["pde"] * V * sum((r * r).sum() for r in R)
    if spec.op == "burgers":
        gx, gt = burgers_smoothing(spec, fine[0])
        terms["reg"] = W["reg"] * V * ((gx * gx).sum() + (gt * gt).sum())
    if spec.op == "heat":
        left, right = heat_boundary(spec, fine[0])
        terms["bc"] = W["bc"] * spec.h[0] * ((left * left).sum() + (right * right).sum())
    for fi, term, idx, vals, wt in spec.meas:
        x = fine[fi].reshape(-1)[torch.as_tensor(idx, dtype=torch.long)]
        d = x - torch.as_tensor(vals, dtype=DT)
        terms[term] = terms[term] + wt * (d * d).sum()
    return terms


def fine_fields(spec, levels):
    """Fine fields u = M_L(levels) for every unknown field."""
    out = []
    for fi, name in enumerate(spec.fields):
        axes = field_axes(spec.op, name, spec.ndim)
        out.append(multigrid.decompose_horner([lv[fi] for lv in levels], axes,
                                              spec.centering))
    return out


def loss_and_grad(spec, levels):
    """Loss terms and the gradient with respect to every level and field.

    levels: list over levels of list over fields (FP64 arrays / tensors).
    Returns (terms: dict of floats, grads: same nesting as levels, float64
    numpy arrays).
    """
    leaves = [[torch.tensor(_np(x), dtype=DT, requires_grad=True) for x in lv]
              for lv in levels]
    fine = fine_fields(spec, leaves)
    terms = loss_terms(spec, fine)
    total = sum(terms.values())
    flat = [x for lv in leaves for x in lv]
    grads = torch.autograd.grad(total, flat, allow_unused=True)
    out, k = [], 0
    for lv in leaves:
        row = []
        for x in lv:
            g = grads[k]
            row.append((torch.zeros_like(x) if g is None else g).detach().numpy())
            k += 1
        out.append(row)
    return {t: float(v.detach()) for t, v in terms.items()}, out


def loss_value(spec, levels):
    with torch.no_grad():
        lv = [[torch.as_tensor(_np(x), dtype=DT) for x in row] for row in levels]
        terms = loss_terms(spec, fine_fields(spec, lv))
    return {t: float(v) for t, v in terms.items()}


def residual_metric(spec, levels):
    """RMS of the cell-integrated PDE residual, sqrt(sum (V R)^2 / count)."""
    with torch.no_grad():
        lv = [[torch.as_tensor(_np(x), dtype=DT) for x in row] for row in levels]
        R = residuals(spec, fine_fields(spec, lv))
        V = spec.cell_measure
        s = math.fsum(float(v) for r in R for v in (V * r).reshape(-1) ** 2)
        count = sum(r.numel() for r in R)
    return math.sqrt(s / count)


def _np(x):
    if isinstance(x, torch.Tensor):
        return x.detach().cpu().to(DT).numpy()
    import numpy as np
    return np.asarray(x, dtype=np.float64)
