"""FP64 oracle of the direct-learning training loop: Adam updates of the TDNN weights
driven by the cascade gradient.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path.

Passages followed:
  * the DPD is trained by gradient descent with the Adam optimiser, learning rate
    0.001, on an MSE loss through the differentiable chain .... Sec. V-A-2
  * the Adam update itself is the one of the cited optimiser paper (Kingma & Ba,
    "Adam: a method for stochastic optimization", Algorithm 1): exponential moving
    averages of the gradient and of its elementwise square, both bias-corrected by
    1 - beta^t, and a step of lr * m_hat / (sqrt(v_hat) + eps).
Default hyper-parameters are that optimiser's (beta1 0.9, beta2 0.999, eps 1e-8);
the paper fixes only the learning rate.  The loss here is the linear NMSE of the
cascade (the readings of dpd_pa.py), so one training step = one full pass over the
given streams (the batch is the whole input).
"""
from __future__ import annotations

import numpy as np

from .dpd_pa import Model, cascade

LR = 1e-3
BETA1 = 0.9
BETA2 = 0.999
EPS = 1e-8


def adam_step(w, m, v, g, t: int, lr: float = LR, beta1: float = BETA1, beta2: float = BETA2,
              eps: float = EPS):
    """One Adam update at step t >= 1 (Algorithm 1 of the optimiser paper), elementwise
    in float64.  Returns new (w, m, v); the inputs are not modified."""
    if t < 1:
        raise ValueError("Adam steps count from 1")
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    w = w - lr * m_hat / (np.sqrt(v_hat) + eps)
    return w, m, v


def train(x_il, offsets, w0, coef, model: Model, steps: int, G: complex = 1.0,
          per_stream: bool = False, lr: float = LR):
    """Direct learning: `steps` Adam updates of the TDNN weights, each from the gradient
    of the pooled linear NMSE of the whole input.  Returns (loss before each step
    [steps][n_sets], final weights shaped like w0)."""
    w = np.asarray(w0, dtype=np.float64).copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    losses = []
    for t in range(1, steps + 1):
        r = cascade(x_il, offsets, w, coef, model, G=G, per_stream=per_stream, grad=True)
        losses.append(r.loss.copy())
        w, m, v = adam_step(w, m, v, r.dw.reshape(w.shape), t, lr=lr)
    return np.array(losses), w
