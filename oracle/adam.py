"""Adam step for the mapping loop, numpy float64.  TEST INFRASTRUCTURE ONLY:
imported by tests, the smoke check and the benchmark's CPU-baseline leg, never
by the product path.

The paper minimises the Eq. (12) loss over the Gaussians' parameters (Sec. II-E)
without naming the optimiser; the Gaussian-splatting lineage it builds on uses
Adam.  This is Adam as Kingma and Ba state it (Algorithm 1 of "Adam: A Method
for Stochastic Optimization", 2015), per parameter element, step t >= 1:
  m <- beta1 m + (1 - beta1) g
  v <- beta2 v + (1 - beta2) g^2
  m_hat = m / (1 - beta1^t),  v_hat = v / (1 - beta2^t)
  p <- p - lr m_hat / (sqrt(v_hat) + eps)
"""
from __future__ import annotations

import numpy as np


def adam_step(p, g, m, v, lr, beta1=0.9, beta2=0.999, eps=1e-15, t=1):
    """Returns the new (p, m, v) as float64 arrays."""
    p, g, m, v = (np.asarray(x, np.float64) for x in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
