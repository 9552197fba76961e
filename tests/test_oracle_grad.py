"""Gradient pins of the FP64 oracle: central finite differences and torch.autograd
(an independent reverse-mode implementation) on tiny shapes.  Follows the
training-by-MSE-through-the-chain setting of Sec. V-A-2."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from dpd_synth import gmp_coefficients, to_interleaved, xavier_tdnn

RNG = np.random.default_rng(99)


def crandn(n, scale=1.0):
    return (RNG.standard_normal(n) + 1j * RNG.standard_normal(n)) * scale / math.sqrt(2)


def tiny_case(T=2, nl=1, H=3, K=3, M=1, L=1, N=32, per_stream=False, S=1, residual=False):
    model = O.Model(T, nl, H, K, M, L, residual)
    lens = [N] if S == 1 else [N, N // 2 + 3, 7][:S]
    x = to_interleaved(crandn(sum(lens))).astype(np.float64)
    off = np.concatenate([[0], np.cumsum(lens)])
    nsets = S if per_stream else 1
    w = np.stack([xavier_tdnn(T, nl, H, seed=4 + s).astype(np.float64) for s in range(nsets)])
    # non-zero biases so that their gradients are exercised
    w += 0.05 * RNG.standard_normal(w.shape)
    coef = np.stack([gmp_coefficients(K, M, L, seed=8 + s).astype(np.float64) for s in range(nsets)])
    if not per_stream:
        w, coef = w[0], coef[0]
    return model, x, off, w, coef


@pytest.mark.parametrize("kw", [
    dict(),
    dict(T=3, nl=2, H=4, K=4, M=2, L=2, N=24),
    dict(residual=True),
    dict(S=3, per_stream=False, N=16),
    dict(S=2, per_stream=True, N=16),
])
def test_gradient_matches_central_differences(kw):
    model, x, off, w, coef = tiny_case(**kw)
    G = 0.9 + 0.2j
    per = kw.get("per_stream", False)
    res = O.cascade(x, off, w, coef, model, G=G, per_stream=per)
    wf = np.array(w, dtype=np.float64)
    shape = wf.shape
    flat = wf.reshape(-1)
    num = np.zeros_like(flat)
    for i in range(flat.size):
        h = 1e-6 * max(1.0, abs(flat[i]))
        wp = flat.copy(); wp[i] += h
        wm = flat.copy(); wm[i] -= h
        lp = O.cascade(x, off, wp.reshape(shape), coef, model, G=G, per_stream=per, grad=False).loss
        lm = O.cascade(x, off, wm.reshape(shape), coef, model, G=G, per_stream=per, grad=False).loss
        num[i] = (lp - lm).sum() / (2 * h)       # each parameter enters one set's loss
    ana = res.dw.reshape(-1)
    rel = np.linalg.norm(ana - num) / np.linalg.norm(num)
    assert rel < 1e-6, rel


def _torch_cascade(x, w, coef, model, G):
    """Independent forward graph in torch float64 (autograd supplies the derivatives)."""
    xr = torch.tensor(x[:, 0], dtype=torch.float64)
    xi = torch.tensor(x[:, 1], dtype=torch.float64)
    xc = torch.complex(xr, xi)
    N = xc.shape[0]
    T, nl, H = model.taps, model.n_hidden, model.hidden
    wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    cols = []
    for t in range(T):
        z = torch.cat([torch.zeros(t, dtype=torch.complex128), xc[:N - t]])
        m = z.abs()
        cols += [z.real, z.imag, m, m ** 2, m ** 3]
    h = torch.stack(cols, 1)
    dims = [5 * T] + [H] * nl + [2]
    pos = 0
    for i in range(len(dims) - 1):
        fi, fo = dims[i], dims[i + 1]
        W = wt[pos:pos + fi * fo].reshape(fo, fi); pos += fi * fo
        b = wt[pos:pos + fo]; pos += fo
        h = h @ W.T + b
        if i < len(dims) - 2:
            h = torch.tanh(h)
    u = torch.complex(h[:, 0], h[:, 1])
    if model.residual:
        u = u + xc
    a, b_, c = O.unpack_gmp(coef, model.K, model.M, model.L)
    a, b_, c = (torch.tensor(v) for v in (a, b_, c))

    def sh(v, d):
        if d >= 0:
            return torch.cat([torch.zeros(d, dtype=v.dtype), v[:N - d]])
        return torch.cat([v[-d:], torch.zeros(-d, dtype=v.dtype)])

    r = u.abs()
    y = torch.zeros(N, dtype=torch.complex128)
    for k in range(model.K):
        for l in range(model.M + 1):
            y = y + a[k, l] * sh(u, l) * sh(r, l) ** k
    for k in range(1, model.K):
        for l in range(model.M + 1):
            for g in range(1, model.L + 1):
                y = y + b_[k - 1, l, g - 1] * sh(u, l) * sh(r, l + g) ** k
                y = y + c[k - 1, l, g - 1] * sh(u, l) * sh(r, l - g) ** k
    e = y - G * xc
    loss = (e.abs() ** 2).sum() / ((G * xc).abs() ** 2).sum()
    loss.backward()
    return loss.item(), wt.grad.numpy(), y.detach().numpy()


@pytest.mark.parametrize("kw", [dict(T=3, nl=2, H=5, K=5, M=3, L=2, N=64),
                                dict(T=4, nl=1, H=6, K=4, M=2, L=1, N=50, residual=True)])
def test_gradient_matches_torch_autograd_fp64(kw):
    model, x, off, w, coef = tiny_case(**kw)
    G = 1.0 + 0.0j
    res = O.cascade(x, off, w, coef, model, G=G)
    loss, g, y = _torch_cascade(x, w, coef, model, G)
    np.testing.assert_allclose(res.y, y, rtol=1e-12, atol=1e-13)
    assert abs(res.loss[0] - loss) <= 1e-12 * loss
    np.testing.assert_allclose(res.dw[0], g, rtol=1e-10, atol=1e-13)


def test_gmp_backward_at_exact_zero_uses_zero_subgradient():
    """d|u|/du at u = 0 is taken as 0 (the choice torch makes for abs)."""
    K, M, L = 3, 1, 1
    coef = gmp_coefficients(K, M, L, seed=1).astype(np.float64)
    a, b, c = O.unpack_gmp(coef, K, M, L)
    u = crandn(10)
    u[4] = 0.0
    g_y = crandn(10)
    g = O.gmp_backward(u, g_y, a, b, c)
    assert np.all(np.isfinite(g))
    # torch on the same graph
    ut = torch.tensor(u, requires_grad=True)
    at, bt, ct = (torch.tensor(v) for v in (a, b, c))
    N = 10

    def sh(v, d):
        if d >= 0:
            return torch.cat([torch.zeros(d, dtype=v.dtype), v[:N - d]])
        return torch.cat([v[-d:], torch.zeros(-d, dtype=v.dtype)])

    r = ut.abs()
    y = torch.zeros(N, dtype=torch.complex128)
    for k in range(K):
        for l in range(M + 1):
            y = y + at[k, l] * sh(ut, l) * sh(r, l) ** k
    for k in range(1, K):
        for l in range(M + 1):
            for gg in range(1, L + 1):
                y = y + bt[k - 1, l, gg - 1] * sh(ut, l) * sh(r, l + gg) ** k
                y = y + ct[k - 1, l, gg - 1] * sh(ut, l) * sh(r, l - gg) ** k
    gy = torch.tensor(g_y)
    # real loss whose real-convention gradient w.r.t. y is g_y: L = Re(sum conj(g_y) y)
    Lr = torch.real(torch.sum(torch.conj(gy) * y))
    Lr.backward()
    # torch returns the conjugate Wirtinger form for complex leaves: grad = dL/dRe + j dL/dIm
    np.testing.assert_allclose(g, ut.grad.numpy(), rtol=1e-12, atol=1e-14)
