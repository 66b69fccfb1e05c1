"""Pins of the Adam oracle (oracle/adam.py): torch.optim.Adam on the CPU in
float64 (a library routine, written in another algebraic form), the first step's
closed form lr g / (|g| + eps), and a zero gradient from zero moments."""
import numpy as np
import torch

from oracle import adam as A


def test_matches_torch_adam_over_steps():
    rng = np.random.default_rng(1)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) * s for s in (1.0, 0.1, 3.0, 0.0, 1e-4)]
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    w = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=lr, betas=(b1, b2), eps=eps)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, start=1):
        w.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = A.adam_step(p, g, m, v, lr, b1, b2, eps, t)
        np.testing.assert_allclose(p, w.detach().numpy(), rtol=0, atol=1e-13)


def test_first_step_closed_form_and_zero_gradient():
    g = np.array([2.0, -0.5, 1e-3, 0.0])
    p, m, v = A.adam_step(np.ones(4), g, np.zeros(4), np.zeros(4), lr=0.01, eps=1e-8, t=1)
    np.testing.assert_allclose(p, 1.0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
    assert p[3] == 1.0
