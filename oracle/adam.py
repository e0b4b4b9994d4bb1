"""Adam update of the learned noise model — TEST INFRASTRUCTURE ONLY.

The learned measurement variance is trained with Adam (Kingma and Ba, 2015,
bias-corrected first and second moments), learning rate 1e-3 and decay rates
0.9 / 0.999.  This is that update written out in float64, one parameter
vector at a time, so that the GPU's training step can be checked against it.
Only the tests may use it.
"""

from __future__ import annotations

import numpy as np


def adam_step(w, m, v, g, step: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam step (step >= 1 counts from the first) on float64 copies of
    the weights w, the moments m and v and the gradient g.  Returns the new
    (w, m, v)."""
    if step < 1:
        raise ValueError("Adam steps count from 1")
    w = np.asarray(w, np.float64)
    g = np.asarray(g, np.float64)
    # exponential moving averages of the gradient and of its square
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * (g * g)
    # both start at zero, so their averages are biased toward zero by the
    # weight (1 - beta^step) that the first `step` terms carry in total
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return w - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
