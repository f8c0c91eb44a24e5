"""The reconstruction studies' own input generators checked against the
oracle (CPU): the Burgers study's reference solution (Section 3.2) is a
discrete solution of the oracle's residual, and its flux is the oracle's."""
import numpy as np
import torch

from oracle import operators as ops
from paper_2303_04679_amd import burgers_study


def test_burgers_study_flux_is_the_oracles():
    rng = np.random.default_rng(3)
    a, b = rng.uniform(-1, 1, 500), rng.uniform(-1, 1, 500)
    got = burgers_study.upwind_flux(a, b)
    want = ops._upwind_flux(torch.tensor(a), torch.tensor(b)).numpy()
    np.testing.assert_allclose(got, want, rtol=1e-15, atol=1e-16)


def test_burgers_study_reference_solves_the_oracles_residual():
    """Every inner point n >= 1, 1 <= i <= N-2 of the study's reference has a
    zero residual of the implicit upwind scheme the oracle evaluates."""
    n = 32
    x = (np.arange(n) + 0.5) / n
    ref = burgers_study.reference(n, x)
    spec = ops.Spec("burgers", (n, n), (1.0, 1.0), 1, weights={"pde": 1.0})
    R = ops.burgers_residual(spec, torch.tensor(ref))[0].numpy()
    scale = np.max(np.abs(ref)) * n
    assert np.max(np.abs(R)) <= 1e-11 * scale, np.max(np.abs(R))
    # the first row is the study's initial condition
    np.testing.assert_allclose(ref[0], 0.5 * (1.0 - np.cos(6.0 * np.pi * x)), rtol=0, atol=1e-15)
