"""Pins of the oracle's ideal linear-clipping PA (the minimum-distortion reference PA of
Sec. V-B-2) and of the cascade through it: closed forms of the definition (identity
below the clipping level, constant envelope with the phase kept above it), brute-force
central differences of its reverse mode, the cascade against the GMP cascade with a
unit-gain PA when nothing clips, and the NMSE and output-bias gradient of a clipped
constant-envelope signal in closed form.  Planted mistakes show that the pins catch
them."""
import math

import numpy as np
import pytest

import oracle as O
import oracle.clip_pa as OCL
from dpd_synth import to_interleaved, xavier_tdnn

RNG = np.random.default_rng(2024)


def crandn(n, scale=1.0):
    return (RNG.standard_normal(n) + 1j * RNG.standard_normal(n)) * scale / math.sqrt(2)


def test_identity_below_clip():
    u = crandn(4000)
    A = 1.01 * np.abs(u).max()
    y = O.clip_forward(u, A)
    assert np.array_equal(y, u)
    # the boundary itself is on the linear branch
    edge = np.array([2.0 + 0j, 0.0 - 2.0j, 2.0 * np.exp(0.3j)])
    assert np.array_equal(O.clip_forward(edge[:2], 2.0), edge[:2])
    assert np.allclose(O.clip_forward(edge[2:], 2.0), edge[2:], rtol=0, atol=1e-15)
    assert O.clip_forward(np.zeros(3, complex), 0.5).tolist() == [0j, 0j, 0j]


def test_constant_envelope_above_clip():
    u = crandn(4000, scale=3.0)
    A = 0.7
    y = O.clip_forward(u, A)
    over = np.abs(u) > A
    assert over.mean() > 0.8
    np.testing.assert_allclose(np.abs(y[over]), A, rtol=1e-15)
    np.testing.assert_allclose(np.angle(y[over]), np.angle(u[over]), rtol=0, atol=1e-14)
    np.testing.assert_array_equal(y[~over], u[~over])
    # the hand-evaluated sample 3 + 4j at A = 1 goes to 0.6 + 0.8j
    np.testing.assert_allclose(O.clip_forward(np.array([3 + 4j]), 1.0), [0.6 + 0.8j], rtol=0, atol=1e-15)


def test_backward_matches_central_differences():
    """L(u) = sum Re(conj(c) y(u)) has g_y = c; its derivatives with respect to Re u and
    Im u of every sample by central differences, on both branches (samples kept away
    from the kink |u| = A)."""
    A = 1.0
    u = crandn(64, scale=1.5)
    u = u[np.abs(np.abs(u) - A) > 0.05]
    c = crandn(u.size)
    assert (np.abs(u) > A).any() and (np.abs(u) <= A).any()

    def loss(v):
        return float(np.sum(np.real(np.conj(c) * O.clip_forward(v, A))))
    h = 1e-7
    num = np.zeros(u.size, dtype=complex)
    for n in range(u.size):
        for step, part in ((h, 1.0), (1j * h, 1j)):
            up = u.copy(); up[n] += step
            um = u.copy(); um[n] -= step
            num[n] += part * (loss(up) - loss(um)) / (2 * h)
    ana = O.clip_backward(u, c, A)
    np.testing.assert_allclose(ana, num, rtol=0, atol=1e-7)


def _tiny(T=2, nl=1, H=3, lens=(40,), per_stream=False, residual=True, seed=3):
    model = O.Model(T, nl, H, 1, 0, 0, residual)
    x = to_interleaved(crandn(sum(lens), scale=1.2)).astype(np.float64)
    off = np.concatenate([[0], np.cumsum(lens)])
    n_sets = len(lens) if per_stream else 1
    w = np.stack([xavier_tdnn(T, nl, H, seed=seed + s).astype(np.float64) for s in range(n_sets)])
    w += 0.05 * RNG.standard_normal(w.shape)
    return model, x, off, (w if per_stream else w[0])


@pytest.mark.parametrize("per_stream", [False, True])
def test_unclipped_cascade_equals_unit_gain_gmp_cascade(per_stream):
    """When A exceeds every |u| the clipping PA is the identity, i.e. the GMP PA with
    K = 1, M = L = 0 and a_00 = 1: same u, y, E, R, loss and gradient."""
    model, x, off, w = _tiny(lens=(30, 17, 5), per_stream=per_stream)
    G = 0.8 - 0.3j
    ref0 = O.cascade(x, off, w, np.tile([[1.0, 0.0]], (3 if per_stream else 1, 1)).reshape(
        (3, 1, 2) if per_stream else (1, 2)), model, G=G, per_stream=per_stream)
    A = 1.5 * np.abs(ref0.u).max()
    got = O.cascade_clip(x, off, w, model, A, G=G, per_stream=per_stream)
    np.testing.assert_array_equal(got.u, ref0.u)
    np.testing.assert_allclose(got.y, ref0.y, rtol=1e-15, atol=0)
    np.testing.assert_allclose(got.E, ref0.E, rtol=1e-13)
    np.testing.assert_allclose(got.loss, ref0.loss, rtol=1e-13)
    np.testing.assert_allclose(got.dw, ref0.dw.reshape(got.dw.shape), rtol=1e-12, atol=1e-15)


def test_clipped_constant_envelope_closed_form():
    """x_n = c e^{j theta_n}, a residual DPD with a zero output layer (u = x), clipping
    level A < c, complex target gain G: y = (A/c) x, so NMSE = |A/c - G|^2 / |G|^2; the
    hidden-layer gradients vanish (the zero output layer passes no delta back) and the
    output-bias gradient is (2 A j Im(A/c - G) / R) sum_n e^{j theta_n}, R = N c^2 |G|^2
    (beyond the clip only the phase of u moves y, so the radial part of the error
    passes nothing)."""
    T, nl, H = 2, 1, 4
    N, c, A, G = 200, 1.7, 1.1, 0.9 + 0.25j
    theta = RNG.uniform(-np.pi, np.pi, N)
    x = c * np.exp(1j * theta)
    model = O.Model(T, nl, H, 1, 0, 0, True)
    w = xavier_tdnn(T, nl, H, seed=7).astype(np.float64)
    n_out = 2 * H + 2
    w[-n_out:] = 0.0
    x_il = np.stack([x.real, x.imag], axis=-1)           # float64, no rounding of x
    res = O.cascade_clip(x_il, [0, N], w, model, A, G=G)
    np.testing.assert_allclose(res.u, x, rtol=0, atol=1e-15)
    np.testing.assert_allclose(res.loss[0], abs(A / c - G) ** 2 / abs(G) ** 2, rtol=1e-13)
    dw = res.dw[0]
    np.testing.assert_array_equal(dw[:-n_out], 0.0)
    R = N * c ** 2 * abs(G) ** 2
    db = 2 * A * 1j * np.imag(A / c - G) / R * np.sum(np.exp(1j * theta))
    np.testing.assert_allclose(dw[-2:], [db.real, db.imag], rtol=1e-12, atol=1e-16)


@pytest.mark.parametrize("per_stream", [False, True])
def test_cascade_gradient_matches_central_differences(per_stream):
    model, x, off, w = _tiny(T=3, nl=2, H=4, lens=(28, 13), per_stream=per_stream)
    G = 0.9 + 0.2j
    base = O.cascade_clip(x, off, w, model, 1e9, G=G, per_stream=per_stream, grad=False)
    r = np.sort(np.abs(base.u))
    k = r.size // 2
    A = float(0.5 * (r[k] + r[k + 1]))              # about half the samples clipped
    assert np.min(np.abs(r - A)) > 1e-6              # no sample at the kink
    res = O.cascade_clip(x, off, w, model, A, G=G, per_stream=per_stream)
    flat = np.array(w, dtype=np.float64).reshape(-1)
    num = np.zeros_like(flat)
    for i in range(flat.size):
        h = 1e-7 * max(1.0, abs(flat[i]))
        wp = flat.copy(); wp[i] += h
        wm = flat.copy(); wm[i] -= h
        lp = O.cascade_clip(x, off, wp.reshape(np.shape(w)), model, A, G=G, per_stream=per_stream,
                            grad=False).loss
        lm = O.cascade_clip(x, off, wm.reshape(np.shape(w)), model, A, G=G, per_stream=per_stream,
                            grad=False).loss
        num[i] = (lp - lm).sum() / (2 * h)
    rel = np.linalg.norm(res.dw.reshape(-1) - num) / np.linalg.norm(num)
    assert rel < 1e-6, rel


# ---------------------------------------------------------------- planted mistakes
def _clip_pins():
    return [test_identity_below_clip, test_constant_envelope_above_clip,
            test_backward_matches_central_differences, test_clipped_constant_envelope_closed_form,
            lambda: test_cascade_gradient_matches_central_differences(False)]


def _caught(monkeypatch, name, replacement):
    monkeypatch.setattr(OCL, name, replacement)
    monkeypatch.setattr(O, name, replacement)
    caught = []
    for pin in _clip_pins():
        try:
            pin()
        except AssertionError:
            caught.append(pin)
    monkeypatch.undo()
    return caught


def test_pins_pass_unmutated():
    for pin in _clip_pins():
        pin()


def _bwd_no_projection(u, g_y, A):
    g = np.array(g_y, dtype=np.complex128)
    over = np.abs(u) > A
    g[over] *= A / np.abs(u[over])
    return g


def _bwd_identity(u, g_y, A):
    return np.array(g_y, dtype=np.complex128)


def _bwd_conjugated(u, g_y, A):
    g = np.array(g_y, dtype=np.complex128)
    r = np.abs(u)
    over = r > A
    v = u[over] / r[over]
    g[over] = (A / r[over]) * (g[over] - v * np.real(v * g[over]))
    return g


def _fwd_scaled_by_square(u, A):
    u = np.asarray(u, dtype=np.complex128)
    r = np.abs(u)
    y = u.copy()
    y[r > A] = A * u[r > A] / r[r > A] ** 2
    return y


def _fwd_clip_at_amplitude_squared(u, A):
    u = np.asarray(u, dtype=np.complex128)
    r = np.abs(u)
    y = u.copy()
    over = r ** 2 > A
    y[over] = A * u[over] / r[over]
    return y


@pytest.mark.parametrize("name,bad", [
    ("clip_backward", _bwd_no_projection), ("clip_backward", _bwd_identity),
    ("clip_backward", _bwd_conjugated), ("clip_forward", _fwd_scaled_by_square),
    ("clip_forward", _fwd_clip_at_amplitude_squared),
])
def test_planted_mistakes_are_caught(monkeypatch, name, bad):
    assert _caught(monkeypatch, name, bad)
