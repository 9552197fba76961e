"""Pins of the FP64 training-loop oracle (oracle/adam.py): the Adam update against its
closed forms and against torch.optim.Adam (an independent implementation of the same
published algorithm), and whole training runs against torch (autograd gradient of an
independent torch graph of the cascade + torch's Adam) on tiny shapes."""
import numpy as np
import pytest
import torch

import oracle.adam as A
from test_oracle_grad import _torch_cascade, tiny_case

RNG = np.random.default_rng(2024)


def test_first_step_moves_by_lr_times_sign():
    """At t = 1 the bias-corrected moments are g and g^2, so the step is lr g / (|g| + eps)."""
    g = RNG.standard_normal(1000) * np.logspace(-6, 2, 1000)
    w0 = RNG.standard_normal(1000)
    w1, m1, v1 = A.adam_step(w0, np.zeros(1000), np.zeros(1000), g, 1)
    np.testing.assert_allclose(w1, w0 - A.LR * g / (np.abs(g) + A.EPS), rtol=1e-14, atol=1e-17)
    np.testing.assert_allclose(m1, (1 - A.BETA1) * g, rtol=1e-15)
    np.testing.assert_allclose(v1, (1 - A.BETA2) * g * g, rtol=1e-15)


def test_constant_gradient_closed_form():
    """With a constant gradient m_hat = g and v_hat = g^2 at every t, so after t steps
    w = w0 - t lr g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, -7e-6])
    w = np.zeros(4); m = np.zeros(4); v = np.zeros(4)
    for t in range(1, 51):
        w, m, v = A.adam_step(w, m, v, g, t, lr=0.01)
        np.testing.assert_allclose(w, -t * 0.01 * g / (np.abs(g) + A.EPS), rtol=1e-12)


def test_matches_torch_adam():
    """A sequence of random gradients (changing scale and sign) through torch.optim.Adam
    in float64 with the same hyper-parameters."""
    n = 257
    w0 = RNG.standard_normal(n)
    grads = [RNG.standard_normal(n) * 10.0 ** RNG.uniform(-4, 1) for _ in range(40)]
    p = torch.nn.Parameter(torch.tensor(w0, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=A.LR, betas=(A.BETA1, A.BETA2), eps=A.EPS)
    w, m, v = w0.copy(), np.zeros(n), np.zeros(n)
    for t, g in enumerate(grads, start=1):
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        w, m, v = A.adam_step(w, m, v, g, t)
        np.testing.assert_allclose(w, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_step_counts_from_one():
    with pytest.raises(ValueError):
        A.adam_step(np.zeros(2), np.zeros(2), np.zeros(2), np.ones(2), 0)


@pytest.mark.parametrize("kw", [dict(T=3, nl=2, H=5, K=5, M=3, L=2, N=64),
                                dict(T=2, nl=1, H=4, K=3, M=1, L=1, N=40, residual=True)])
def test_training_run_matches_torch(kw):
    """Six direct-learning steps: the oracle's loss trajectory and final weights against
    torch autograd on an independent graph of the cascade, stepped by torch's Adam
    (learning rate 0.01 so the weights move visibly)."""
    model, x, off, w, coef = tiny_case(**kw)
    steps, lr = 6, 1e-2
    losses, w_or = A.train(x, off, w, coef, model, steps, lr=lr)
    p = torch.nn.Parameter(torch.tensor(w, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=lr, betas=(A.BETA1, A.BETA2), eps=A.EPS)
    ref_losses = []
    for _ in range(steps):
        loss, g, _ = _torch_cascade(x, p.detach().numpy(), coef, model, 1.0 + 0.0j)
        ref_losses.append(loss)
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(losses[:, 0], ref_losses, rtol=1e-10)
    np.testing.assert_allclose(w_or, p.detach().numpy(), rtol=1e-9, atol=1e-12)
    assert losses[-1, 0] < losses[0, 0]          # the steps descend


def _mutant(kind):
    def step(w, m, v, g, t, lr=A.LR, beta1=A.BETA1, beta2=A.BETA2, eps=A.EPS):
        m = beta1 * m + ((1 - beta2) if kind == "m_rate" else (1 - beta1)) * g
        v = beta2 * v + (1 - beta2) * g * g
        c1 = 1.0 if kind == "no_bias_corr" else 1 - beta1 ** t
        c2 = 1.0 if kind == "no_bias_corr" else 1 - (beta1 if kind == "v_corr_beta1" else beta2) ** t
        den = np.sqrt(v / c2 + eps) if kind == "eps_in_sqrt" else np.sqrt(v / c2) + eps
        sign = -1.0 if kind == "ascent" else 1.0
        return w - sign * lr * (m / c1) / den, m, v
    return step


@pytest.mark.parametrize("kind", ["m_rate", "no_bias_corr", "v_corr_beta1", "eps_in_sqrt", "ascent"])
def test_planted_adam_mistakes_are_caught(monkeypatch, kind):
    monkeypatch.setattr(A, "adam_step", _mutant(kind))
    pins = [test_first_step_moves_by_lr_times_sign, test_constant_gradient_closed_form,
            test_matches_torch_adam,
            lambda: test_training_run_matches_torch(dict(T=2, nl=1, H=4, K=3, M=1, L=1, N=40))]
    caught = 0
    for p in pins:
        try:
            p()
        except AssertionError:
            caught += 1
    assert caught > 0
