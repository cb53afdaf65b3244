"""The Adam update from its definition (Kingma and Ba), in FP64.

The paper does not name its optimiser; 3DGS-family training uses Adam, with
bias correction and per-parameter-group learning rates:

  m <- b1 m + (1 - b1) g
  v <- b2 v + (1 - b2) g^2
  p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
"""
import numpy as np


def adam_step(p, g, m, v, lr, b1, b2, eps, step):
    p = np.asarray(p, np.float64).copy()
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    p -= lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v
