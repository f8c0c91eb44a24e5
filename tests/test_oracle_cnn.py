"""Pins of the warm-start network reference."""
import numpy as np
import torch

from oracle import cnn


def test_bf16_rounding_ties_to_even():
    e = 2.0 ** -8
    x = np.array([1.0 + e, 1.0 + 3 * e, 1.0 + 1.01 * e, -(1.0 + e), 3.0], dtype=np.float32)
    r = cnn.bf16_round(x).numpy()
    np.testing.assert_array_equal(r, [1.0, 1.0 + 4 * e, 1.0 + 2 * e, -1.0, 3.0])


def test_output_shapes():
    specs = cnn.layer_specs(5, 6, 7, 3)
    th = torch.zeros(cnn.n_params(specs), dtype=torch.float64)
    act, out = cnn.forward(th, specs, np.zeros((2, 4, 32, 32)))
    assert out.shape == (2, 3 * (8 * 8 + 4 * 4 + 2 * 2))
    assert act.shape == (2, 5 * 64 + 6 * 16 + 7 * 4)


def test_gradient_matches_central_differences():
    specs = cnn.layer_specs(2, 3, 3, 3)
    rng = np.random.default_rng(0)
    th = rng.normal(0, 0.5, cnn.n_params(specs))
    img = rng.normal(0, 1, (2, 4, 16, 16))
    tgt = rng.normal(0, 1, (2, 3 * (16 + 4 + 1)))
    loss, g = cnn.loss_and_grad(th, specs, img, tgt)
    fd = np.zeros_like(th)
    for k in range(th.size):
        x0 = th[k]
        th[k] = x0 + 1e-6
        lp, _ = cnn.loss_and_grad(th, specs, img, tgt)
        th[k] = x0 - 1e-6
        lm, _ = cnn.loss_and_grad(th, specs, img, tgt)
        th[k] = x0
        fd[k] = (lp - lm) / 2e-6
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < 1e-6


def test_rasterize():
    img = cnn.rasterize(4, [np.array([1, 6])], [np.array([0.5, -1.0])], [np.array([2.0, 3.0])],
                        [775.0], 550.0, 450.0)
    assert img[0, 0].ravel()[1] == 0.5 and img[0, 1].ravel()[6] == 3.0
    assert img[0, 2].sum() == 2.0 and np.all(img[0, 3] == 0.5)
