"""Adam update (Kingma & Ba; the optimiser the paper runs in Section 2.1, 3.1).

The paper does not print its hyper-parameters.  The reading used here is the
textbook algorithm with the bias corrections and epsilon added to the square
root of the corrected second moment:

    m <- b1 m + (1 - b1) g
    v <- b2 v + (1 - b2) g^2
    theta <- theta - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

with the step counter t starting at 1.  All levels and fields share lr.
"""
import numpy as np


def adam_step(theta, m, v, g, lr, beta1, beta2, eps, t):
    """One Adam step in FP64; returns (theta, m, v) as new arrays."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v
