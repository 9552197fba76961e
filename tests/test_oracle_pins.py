"""Pins of the FP64 oracle against values fixed independently of it.

Each test names the passage of arXiv 2205.05158 it checks.  A plausible mistake in
the oracle (a dropped GMP family, lag/lead swapped, a wrong tap index, a
transposed weight matrix, a wrong NMSE normalisation) fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.signal

import oracle as O
from dpd_synth import (gmp_coeff_count, gmp_coefficients, ofdm_signal, to_interleaved,
                       xavier_tdnn)

RNG = np.random.default_rng(1234)


def crandn(n, rng=RNG, scale=1.0):
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * scale / math.sqrt(2)


def packed_gmp(K, M, L, a=None, b=None, c=None):
    a = np.zeros((K, M + 1), complex) if a is None else a
    b = np.zeros((K - 1, M + 1, L), complex) if b is None else b
    c = np.zeros((K - 1, M + 1, L), complex) if c is None else c
    z = np.concatenate([a.ravel(), b.ravel(), c.ravel()])
    return np.stack([z.real, z.imag], axis=1)          # float64, no float32 rounding


# ---------------------------------------------------------------- GMP, eq. (9)
def test_gmp_linear_gain_only():
    """Only a_{0,0} = alpha: eq. (9) reduces to y = alpha * u (k = 0, l = 0 term)."""
    K, M, L = 5, 3, 2
    alpha = 0.7 - 0.2j
    a = np.zeros((K, M + 1), complex)
    a[0, 0] = alpha
    u = crandn(257)
    y = O.gmp_forward(u, *O.unpack_gmp(packed_gmp(K, M, L, a=a), K, M, L))
    np.testing.assert_allclose(y, alpha * u, rtol=0, atol=1e-15)


def test_gmp_fir_matches_numpy_convolve():
    """Only a_{0,l}: eq. (9) is the causal FIR sum_l a_{0,l} u[n-l] (np.convolve)."""
    K, M, L = 3, 4, 2
    a = np.zeros((K, M + 1), complex)
    a[0, :] = crandn(M + 1)
    u = crandn(300)
    y = O.gmp_forward(u, *O.unpack_gmp(packed_gmp(K, M, L, a=a), K, M, L))
    np.testing.assert_allclose(y, np.convolve(u, a[0])[:u.size], rtol=0, atol=1e-13)


def test_gmp_memoryless_constant_envelope_closed_form():
    """M = 0, L = 0: y = u * p(|u|), p(A) = sum_k a_k A^k.  For a constant-envelope input
    A e^{j w n} the NMSE against G x is |p(A) - G|^2 / |G|^2 in closed form."""
    K = 6
    a = crandn(K).reshape(K, 1)
    A, w, G = 1.3, 0.37, 0.9 + 0.1j
    n = np.arange(500)
    x = A * np.exp(1j * w * n)
    y = O.gmp_forward(x, a, np.zeros((K - 1, 1, 0), complex), np.zeros((K - 1, 1, 0), complex))
    p = sum(a[k, 0] * A ** k for k in range(K))
    np.testing.assert_allclose(y, x * p, rtol=1e-13)
    E, R = O.nmse_parts(y, x, G)
    np.testing.assert_allclose(E / R, abs(p - G) ** 2 / abs(G) ** 2, rtol=1e-12)


def test_gmp_lag_term_direction():
    """A single b_{k=1,l=0,g=1}: y[n] = b u[n] |u[n-1]|, the envelope is delayed (lag)."""
    K, M, L = 3, 2, 2
    b = np.zeros((K - 1, M + 1, L), complex)
    b[0, 0, 0] = 0.5 + 0.25j
    u = crandn(64)
    y = O.gmp_forward(u, *O.unpack_gmp(packed_gmp(K, M, L, b=b), K, M, L))
    expect = np.zeros_like(u)
    for n in range(u.size):
        expect[n] = b[0, 0, 0] * u[n] * (abs(u[n - 1]) if n >= 1 else 0.0)
    np.testing.assert_allclose(y, expect, rtol=1e-14, atol=1e-15)


def test_gmp_lead_term_direction():
    """A single c_{k=2,l=1,g=2}: y[n] = c u[n-1] |u[n+1]|^2 (lead, inside the stream only)."""
    K, M, L = 4, 2, 2
    c = np.zeros((K - 1, M + 1, L), complex)
    c[1, 1, 1] = -0.3 + 0.8j
    u = crandn(50)
    N = u.size
    y = O.gmp_forward(u, *O.unpack_gmp(packed_gmp(K, M, L, c=c), K, M, L))
    expect = np.zeros_like(u)
    for n in range(N):
        up = u[n - 1] if n >= 1 else 0.0
        rq = abs(u[n + 1]) if n + 1 < N else 0.0
        expect[n] = c[1, 1, 1] * up * rq ** 2
    np.testing.assert_allclose(y, expect, rtol=1e-14, atol=1e-14)


def test_gmp_brute_force_tiny():
    """All families at once vs a scalar loop over n, k, l, g with explicit indices."""
    K, M, L = 4, 2, 2
    coef = gmp_coefficients(K, M, L, seed=7).astype(np.float64)
    a, b, c = O.unpack_gmp(coef, K, M, L)
    u = crandn(23)
    N = u.size

    def U(i):
        return u[i] if 0 <= i < N else 0.0

    expect = np.zeros(N, complex)
    for n in range(N):
        s = 0.0
        for k in range(K):
            for l in range(M + 1):
                s += a[k, l] * U(n - l) * abs(U(n - l)) ** k
        for k in range(1, K):
            for l in range(M + 1):
                for g in range(1, L + 1):
                    s += b[k - 1, l, g - 1] * U(n - l) * abs(U(n - l - g)) ** k
                    s += c[k - 1, l, g - 1] * U(n - l) * abs(U(n - l + g)) ** k
        expect[n] = s
    np.testing.assert_allclose(O.gmp_forward(u, a, b, c), expect, rtol=1e-13, atol=1e-14)


def test_gmp_least_squares_identification():
    """y is linear in the J coefficients; building the basis matrix column by column
    from unit coefficient vectors and solving least squares recovers the generating
    coefficients (the LS identification of Sec. V-A-2)."""
    K, M, L = 4, 2, 1
    J = gmp_coeff_count(K, M, L)
    true = gmp_coefficients(K, M, L, seed=11).astype(np.float64)
    u = crandn(400)
    cols = []
    for j in range(J):
        e = np.zeros((J, 2))
        e[j, 0] = 1.0
        cols.append(O.gmp_forward(u, *O.unpack_gmp(e, K, M, L)))
    Phi = np.stack(cols, axis=1)
    y = O.gmp_forward(u, *O.unpack_gmp(true, K, M, L))
    est, *_ = np.linalg.lstsq(Phi, y, rcond=None)
    np.testing.assert_allclose(est, true[:, 0] + 1j * true[:, 1], atol=1e-9)
    # every basis column is non-trivial: no monomial silently dropped
    assert np.all(np.linalg.norm(Phi, axis=0) > 0)
    assert np.linalg.matrix_rank(Phi) == J


def test_gmp_term_count_matches_eq9():
    """eq. (9) has K(L3+1) + 2(K-1)(L3+1)G monomials."""
    for K, M, L in [(5, 3, 2), (7, 5, 3), (9, 7, 4), (7, 3, 1)]:
        assert len(O.gmp_terms(K, M, L)) == gmp_coeff_count(K, M, L)
    assert gmp_coeff_count(7, 3, 1) == 76          # the paper's PA / TD-GMP setting


# ------------------------------------------------------ target and NMSE, Sec. II-B
def test_linear_pa_identity_dpd_zero_error():
    """Linear PA (a_{0,0} = G, rest 0) after an identity DPD (residual TDNN with zero
    output layer) gives y = G x exactly: E = 0, NMSE = -inf dB."""
    T, nl, H, K, M, L = 3, 2, 5, 4, 2, 2
    G = 1.0 + 0.0j
    w = xavier_tdnn(T, nl, H, seed=3).astype(np.float64)
    layers = O.unpack_tdnn(w, T, nl, H)
    layers[-1] = (np.zeros_like(layers[-1][0]), np.zeros(2))
    w = O.pack_tdnn(layers)
    a = np.zeros((K, M + 1), complex)
    a[0, 0] = G
    coef = packed_gmp(K, M, L, a=a)
    xc = crandn(200)
    x = np.stack([xc.real, xc.imag], axis=1)
    res = O.cascade(x, [0, 200], w, coef, O.Model(T, nl, H, K, M, L, residual=True), G=G)
    np.testing.assert_array_equal(res.y, O.complex_of(x) * G)
    assert res.E[0] == 0.0 and O.db10(res.E[0] / res.R[0]) == float("-inf")


@pytest.mark.parametrize("delta", [0.1, 0.01, 1e-3])
def test_nmse_scaled_target(delta):
    """y = (1 + delta) G x  =>  NMSE_dB = 20 log10 |delta|."""
    x = crandn(1000)
    G = 0.8 - 0.3j
    E, R = O.nmse_parts((1 + delta) * G * x, x, G)
    assert abs(10 * math.log10(E / R) - 20 * math.log10(delta)) < 1e-9


# ------------------------------------------------------ TDNN (Sec. III-C core, eq. (8))
def test_features_exact_values_and_taps():
    """Features of tap t are (Re, Im, |.|, |.|^2, |.|^3) of x[n-t], zero before the stream."""
    x = np.array([3 + 4j, -1 + 0j, 0 + 2j, 1 - 1j])
    F = O.features(x, 3)
    assert F.shape == (4, 15)
    np.testing.assert_array_equal(F[0, 0:5], [3, 4, 5, 25, 125])
    np.testing.assert_array_equal(F[0, 5:15], 0)               # no samples before n = 0
    np.testing.assert_array_equal(F[2, 5:10], [-1, 0, 1, 1, 1])  # tap 1 of n = 2 is x[1]
    np.testing.assert_array_equal(F[3, 10:15], [-1, 0, 1, 1, 1])  # tap 2 of n = 3 is x[1]
    np.testing.assert_allclose(F[3, 0:5], [1, -1, math.sqrt(2), 2, 2 * math.sqrt(2)], rtol=1e-15)


def test_tdnn_hand_evaluated_single_neuron():
    """T = 1, one hidden layer of one neuron: u = wo0 tanh(v.phi + b1) + bo0
    + j (wo1 tanh(...) + bo1), evaluated by hand."""
    v = np.array([0.1, -0.2, 0.3, 0.05, -0.01])
    b1 = 0.2
    wo = np.array([[1.5], [-0.5]])
    bo = np.array([0.1, 0.3])
    w = np.concatenate([v, [b1], wo.ravel(), bo])
    layers = O.unpack_tdnn(w, 1, 1, 1)
    x = np.array([0.6 - 0.8j])                      # |x| = 1
    u, _ = O.tdnn_forward(x, layers)
    t = math.tanh(0.1 * 0.6 + (-0.2) * (-0.8) + 0.3 * 1 + 0.05 * 1 + (-0.01) * 1 + 0.2)
    assert abs(u[0] - ((1.5 * t + 0.1) + 1j * (-0.5 * t + 0.3))) < 1e-15


def test_tdnn_weight_orientation():
    """W is [fan_out][fan_in] (rows are output neurons): a one-hot W1 picks exactly the
    named feature; the transposed reading would pick another."""
    T, H = 2, 3
    w = np.zeros(H * 10 + H + H * 2 + 2)
    layers = O.unpack_tdnn(w, T, 1, H)
    W1 = layers[0][0].copy()
    W1[2, 8] = 1.0                                   # neuron 2 reads feature 8 = |x[n-1]|^2
    Wo = layers[1][0].copy()
    Wo[0, 2] = 1.0
    layers = [(W1, layers[0][1]), (Wo, layers[1][1])]
    x = np.array([0.0, 0.5j, 0.3 + 0.4j])
    u, _ = O.tdnn_forward(x, layers)
    np.testing.assert_allclose(u.real, np.tanh([0.0, 0.0, 0.25]), rtol=1e-15)
    np.testing.assert_allclose(u.imag, 0.0)


def test_stream_start_equals_zero_prefix():
    """Zero padding at a stream start: outputs equal those of the same stream with an
    explicit zero prefix, for the TDNN (tap window) and the whole cascade except where
    the GMP lead terms would see the prefix."""
    T, nl, H, K, M, L = 4, 2, 6, 5, 3, 2
    w = xavier_tdnn(T, nl, H, seed=5).astype(np.float64)
    layers = O.unpack_tdnn(w, T, nl, H)
    x = crandn(40)
    u, _ = O.tdnn_forward(x, layers)
    up, _ = O.tdnn_forward(np.concatenate([np.zeros(T - 1), x]), layers)
    np.testing.assert_allclose(u, up[T - 1:], rtol=1e-14, atol=1e-15)


def test_batched_streams_equal_separate_streams():
    """Independent streams: running them together equals running each alone."""
    T, nl, H, K, M, L = 3, 2, 7, 4, 2, 2
    model = O.Model(T, nl, H, K, M, L)
    lens = [37, 5, 64]
    xs = [to_interleaved(crandn(n)).astype(np.float64) for n in lens]
    ws = [xavier_tdnn(T, nl, H, seed=s).astype(np.float64) for s in range(3)]
    cs = [gmp_coefficients(K, M, L, seed=10 + s).astype(np.float64) for s in range(3)]
    off = np.concatenate([[0], np.cumsum(lens)])
    res = O.cascade(np.concatenate(xs), off, np.stack(ws), np.stack(cs), model, per_stream=True)
    for s in range(3):
        one = O.cascade(xs[s], [0, lens[s]], ws[s], cs[s], model)
        np.testing.assert_allclose(res.y[off[s]:off[s + 1]], one.y, rtol=1e-14, atol=1e-14)
        np.testing.assert_allclose(res.dw[s], one.dw[0], rtol=1e-12, atol=1e-14)
        assert abs(res.loss[s] - one.loss[0]) <= 1e-14 * one.loss[0]


def test_cascade_at_matches_full_stream():
    """Windowed single-output evaluation equals the full-stream forward, including both
    stream edges."""
    T, nl, H, K, M, L = 4, 2, 5, 5, 3, 2
    model = O.Model(T, nl, H, K, M, L)
    x = to_interleaved(crandn(120)).astype(np.float64)
    w = xavier_tdnn(T, nl, H, seed=2).astype(np.float64)
    coef = gmp_coefficients(K, M, L, seed=3).astype(np.float64)
    full = O.cascade(x, [0, 120], w, coef, model, grad=False)
    idx = np.array([0, 1, 2, 7, 60, 117, 118, 119])
    u, y = O.cascade_at(x, idx, w, coef, model)
    np.testing.assert_allclose(u, full.u[idx], rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(y, full.y[idx], rtol=1e-13, atol=1e-14)


# ------------------------------------------------------ Welch PSD / ACPR
def test_psd_matches_scipy_welch():
    y = crandn(4096 * 5 + 123)
    ours = O.welch_psd(y, 4096)
    _, ref = scipy.signal.welch(y, fs=1.0, window="hann", nperseg=4096, noverlap=2048,
                                detrend=False, return_onesided=False, scaling="density")
    np.testing.assert_allclose(ours, ref, rtol=1e-10)


def test_psd_parseval_and_tone_bin():
    """mean(PSD) equals the mean power for a tone on a bin centre; the tone's power
    lands in its own bin and the two Hann neighbours (weights 1, 1/4, 1/4)."""
    nfft = 1024
    k0 = 100
    n = np.arange(nfft * 8)
    y = 2.0 * np.exp(2j * np.pi * k0 * n / nfft)
    psd = O.welch_psd(y, nfft)
    np.testing.assert_allclose(psd.mean(), 4.0, rtol=1e-12)
    ratio = psd[k0 - 1:k0 + 2] / psd[k0]
    np.testing.assert_allclose(ratio, [0.25, 1.0, 0.25], rtol=1e-10)
    assert psd[k0 + 2:].max() < 1e-20 * psd[k0]


def test_acpr_grows_with_third_order_distortion():
    """Third-order distortion x|x|^2 spreads power into the adjacent channels (spectral
    regrowth), so ACPR rises monotonically with its strength.  The undistorted signal's
    floor comes from the symbol-boundary discontinuities (no cyclic prefix)."""
    x = ofdm_signal(4096, 1024, 24, 64, np.random.default_rng(0))
    vals = [O.acpr_db(O.welch_psd(x + a * x * np.abs(x) ** 2, 4096), 512)[2]
            for a in (0.0, 0.05, 0.2, 0.5)]
    assert vals[0] < -25
    assert all(v1 > v0 + 0.5 for v0, v1 in zip(vals, vals[1:]))
    psd = O.welch_psd(x, 4096)
    lo, mn, up = O.band_powers(psd, 512)
    assert 0.999 < (lo + mn + up) / psd.sum() <= 1.0


# ACPR channel plan (the reading of the ACPR the paper names in Sec. I without an
# estimator): main channel |k| <= h, upper adjacent h < k <= 3h, lower -3h <= k < -h.
# These pins fix each edge and the side of each adjacent channel with hand-built inputs.
def _bands_of_single_bin(k, nfft, h):
    import oracle.spectrum as OS
    psd = np.zeros(nfft)
    psd[k % nfft] = 1.0
    return OS.band_powers(psd, h)


@pytest.mark.parametrize("k,band", [
    (0, "M"), (7, "M"), (20, "M"), (-20, "M"),           # |k| <= h (h = 20), DC included
    (21, "U"), (40, "U"), (60, "U"),                      # h < k <= 3h
    (-21, "L"), (-40, "L"), (-60, "L"),                   # -3h <= k < -h
    (61, None), (-61, None), (127, None), (-128, None),   # beyond 3h: no channel
])
def test_band_plan_single_bin_membership(k, band):
    """Unit power in one PSD bin lands in exactly the channel the plan assigns."""
    lo, mn, up = _bands_of_single_bin(k, 256, 20)
    expect = {"L": (1.0, 0.0, 0.0), "M": (0.0, 1.0, 0.0), "U": (0.0, 0.0, 1.0), None: (0.0, 0.0, 0.0)}[band]
    assert (lo, mn, up) == expect


def test_band_plan_exact_sums_of_distinct_bins():
    """Every bin carries a distinct power of two, so each channel sum identifies the exact
    set of bins it took: main = bins -h..h, upper = h+1..3h, lower = -3h..-h-1."""
    import oracle.spectrum as OS
    nfft, h = 64, 5
    ks = np.where(np.arange(nfft) < nfft // 2, np.arange(nfft), np.arange(nfft) - nfft)
    psd = 2.0 ** (ks + 32)                                   # exact in float64
    lo, mn, up = OS.band_powers(psd, h)
    assert mn == sum(2.0 ** (k + 32) for k in range(-h, h + 1))
    assert up == sum(2.0 ** (k + 32) for k in range(h + 1, 3 * h + 1))
    assert lo == sum(2.0 ** (k + 32) for k in range(-3 * h, -h))


def test_acpr_of_tones_in_known_channels():
    """Tones on bin centres: a unit tone at DC (main), one of power 1e-2 at k = 5h/2
    (upper adjacent, beyond 2h) and one of power 1e-4 at k = -5h/2 (lower).  Each tone's
    Hann leakage (bins k0 - 1, k0, k0 + 1) stays inside its channel, so ACPR_U = -20 dB and
    ACPR_L = -40 dB exactly (up to rounding): pins the sides of L and U and the 2h width."""
    import oracle.spectrum as OS
    nfft, h = 1024, 40
    n = np.arange(nfft * 6)
    y = (1.0 + 0.1 * np.exp(2j * np.pi * (5 * h // 2) * n / nfft)
         + 0.01 * np.exp(-2j * np.pi * (5 * h // 2) * n / nfft))
    aL, aU, amax = OS.acpr_db(OS.welch_psd(y, nfft), h)
    np.testing.assert_allclose([aL, aU, amax], [-40.0, -20.0, -20.0], atol=1e-9)
