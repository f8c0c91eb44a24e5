"""Pins of the oracle's gradient and optimiser.

* central finite differences of the loss, every parameter of every level
* torch.optim.Adam (a library routine) for the update
* method-level invariants from the paper: L = 1 is plain ODIL (Section 3.1),
  the fine-field trajectory does not depend on how the initial field is split
  over levels, and more levels converge faster on the Poisson problem
"""
import numpy as np
import pytest
import torch

from oracle import adam as oadam
from oracle import multigrid as mg
from oracle import operators as ops
from tests.oracle_cases import case, random_levels

CASES = [
    ("poisson", (8,), 3),
    ("poisson_node", (8,), 3),
    ("poisson_node", (8, 4), 2),
    ("poisson_node", (4, 4, 4), 2),
    ("poisson", (8, 8), 3),
    ("poisson", (4, 4, 4), 2),
    ("burgers", (8, 8), 3),
    ("heat", (8, 8), 3),
    ("ns3d", (4, 4, 4), 2),
    ("ns3d_fixed", (4, 4, 4), 2),
    ("ns3d_node", (4, 4, 4), 2),
    ("ns3d_fixed_node", (4, 2, 4), 2),
    ("cavity", (8, 8), 3),
    ("cavity_node", (8, 8), 3),
    ("cavity_node", (8, 4), 2),
]


def _total(spec, levels):
    return sum(ops.loss_value(spec, levels).values())


@pytest.mark.parametrize("op,dims,L", CASES)
def test_gradient_matches_central_differences(op, dims, L):
    spec = case(op, dims, L, seed=3, with_forcing=op != "poisson")
    levels = random_levels(spec, seed=4)
    if op == "burgers":   # keep away from the kink of |mean| in the upwind flux
        levels = random_levels(spec, seed=4, lo=0.2, hi=1.0)
    terms, grads = ops.loss_and_grad(spec, levels)
    for li, row in enumerate(levels):
        for fi, arr in enumerate(row):
            fd = np.zeros_like(arr)
            for k in range(arr.size):
                x0 = arr.flat[k]
                step = 1e-6 * max(1.0, abs(x0))
                arr.flat[k] = x0 + step
                lp = _total(spec, levels)
                arr.flat[k] = x0 - step
                lm = _total(spec, levels)
                arr.flat[k] = x0
                fd.flat[k] = (lp - lm) / (2 * step)
            g = grads[li][fi]
            err = np.linalg.norm(g - fd) / max(np.linalg.norm(fd), 1e-30)
            assert err < 2e-6, (op, li, fi, err)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    p = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 21):
        g = rng.standard_normal(50) * (t % 3 + 0.1)
        theta, m, v = oadam.adam_step(theta, m, v, g, 1e-3, 0.9, 0.999, 1e-8, t)
        p.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(theta, p.detach().numpy(), rtol=0, atol=1e-14)


def test_single_level_is_plain_odil():
    """With L = 1 the decomposition is the identity: the loss is that of the grid field."""
    spec = case("cavity", (8, 8), 1, seed=1)
    levels = random_levels(spec, seed=2)
    terms, grads = ops.loss_and_grad(spec, levels)
    fine = [torch.tensor(x) for x in levels[0]]
    direct = ops.loss_terms(spec, fine)
    for t in terms:
        assert terms[t] == float(direct[t])


def _adam_fine_trajectory(spec, levels, steps, lr):
    state = [[(x.copy(), np.zeros_like(x), np.zeros_like(x)) for x in row] for row in levels]
    for t in range(1, steps + 1):
        cur = [[s[0] for s in row] for row in state]
        _, grads = ops.loss_and_grad(spec, cur)
        state = [[oadam.adam_step(s[0], s[1], s[2], g, lr, 0.9, 0.999, 1e-8, t)
                  for s, g in zip(row, grow)] for row, grow in zip(state, grads)]
    cur = [[s[0] for s in row] for row in state]
    with torch.no_grad():
        return [f.numpy() for f in ops.fine_fields(spec, [[torch.tensor(x) for x in r] for r in cur])]


def test_decomposition_invariance():
    """Adam's update depends on gradients only, and dL/du_l = P_l^T g(M u): the
    fine-field trajectory is the same whether a constant initial field sits on
    the finest or the coarsest level."""
    spec = case("poisson", (16, 16), 4, seed=5)
    shapes = ops.level_shapes("poisson", spec.dims, 4)
    a = [[np.zeros(s[0])] for s in shapes]
    b = [[np.zeros(s[0])] for s in shapes]
    a[0][0][:] = 0.3
    b[-1][0][:] = 0.3        # T reproduces constants, so M gives the same fine field
    fa = _adam_fine_trajectory(spec, a, 15, 1e-2)
    fb = _adam_fine_trajectory(spec, b, 15, 1e-2)
    np.testing.assert_allclose(fa[0], fb[0], rtol=0, atol=1e-12)


def test_more_levels_converge_faster_poisson_adam():
    """Section 3.1: increasing the number of levels accelerates Adam (loose check)."""
    from oracle import reference as ref
    n = 16
    errs = {}
    for L in (1, 3):
        spec = ops.Spec("poisson", (n, n), (1.0, 1.0), L, weights={"pde": 1.0})
        u_ref = ref.poisson_reference((n, n))
        spec.forcing = {0: ref.poisson_forcing(spec, u_ref)}
        shapes = ops.level_shapes("poisson", spec.dims, L)
        lv = [[np.zeros(s[0])] for s in shapes]
        fine = _adam_fine_trajectory(spec, lv, 100, 5e-3)
        errs[L] = np.sqrt(np.mean((fine[0] - u_ref) ** 2))
    assert errs[3] < 0.8 * errs[1], errs
