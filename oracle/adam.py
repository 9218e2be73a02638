"""Adam, as the optimiser of the critic and actor updates, in FP64 numpy.

Algorithm 1 writes the critic and policy updates as gradient steps with a
learning rate and names no optimiser; the readings here are Adam
(Kingma & Ba, 2015, Algorithm 1) with beta1 = 0.9, beta2 = 0.999,
eps = 1e-8 added outside the square root, bias correction with the step
number t >= 1, and no weight decay (Appendix E reports weight decay did not
help).  Learning rates follow the hyperparameter table (critic 3e-4,
policy 6e-4).

Test infrastructure only (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import numpy as np


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9,
              b2: float = 0.999, eps: float = 1e-8):
    """Returns updated (p, m, v) for step number t (t >= 1)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
