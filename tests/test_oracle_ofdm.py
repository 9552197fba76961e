"""Pins of the downlink oracle (FD-NN wrapper, ZF precoding, cyclic GMP, QAM decisions,
link) against definitions written out independently, closed forms and invariants."""
import math

import numpy as np
import pytest

import dpd_synth as syn
from oracle import dpd_pa, ofdm


def _c(a):
    return a[..., 0].astype(np.float64) + 1j * a[..., 1].astype(np.float64)


def _rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------------------
# DFT pair
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N", [1, 2, 8, 12])
def test_dft_is_the_unitary_sum(N):
    rng = np.random.default_rng(N)
    x = _rand_c(rng, 3, N)
    X = np.zeros_like(x)
    for k in range(N):
        for n in range(N):
            X[:, k] += x[:, n] * complex(math.cos(2 * math.pi * k * n / N), -math.sin(2 * math.pi * k * n / N))
    X /= math.sqrt(N)
    np.testing.assert_allclose(ofdm.dft(x), X, atol=1e-12)
    # eq. (2): the inverse carries the + sign and the same 1/sqrt(N)
    xi = np.zeros_like(x)
    for n in range(N):
        for k in range(N):
            xi[:, n] += X[:, k] * complex(math.cos(2 * math.pi * k * n / N), math.sin(2 * math.pi * k * n / N))
    np.testing.assert_allclose(ofdm.idft(X), xi / math.sqrt(N), atol=1e-12)
    np.testing.assert_allclose(ofdm.idft(ofdm.dft(x)), x, atol=1e-12)
    np.testing.assert_allclose(np.sum(np.abs(X) ** 2), np.sum(np.abs(x) ** 2), rtol=1e-12)


def test_data_bins():
    b = ofdm.data_bins(64, 16)
    assert b.size == 16 and len(set(b.tolist())) == 16 and 0 not in b
    assert b.tolist() == list(range(1, 9)) + list(range(56, 64))
    # the generator places data symbol d on the same subcarrier
    idx, s = syn.downlink_symbols(2, 3, 64, 16, 16, 5)
    S = _c(s)
    pts = ofdm.qam_points(16)
    np.testing.assert_allclose(S[:, :, b], pts[idx], atol=1e-6)
    guard = np.setdiff1d(np.arange(64), b)
    assert np.all(S[:, :, guard] == 0)


# ---------------------------------------------------------------------------
# FD-NN
# ---------------------------------------------------------------------------
def _brute_fdnn(S, w, U, L4, D, nh):
    """Per-sample, per-neuron loops with explicit DFT sums (tiny sizes only)."""
    n_sym, _, N = S.shape
    F = 2 * U * (L4 + 1)
    w = np.asarray(w, dtype=np.float64)
    pos = 0
    mats = []
    for fi, fo in [(F, D)] + [(D, D)] * (nh - 1) + [(D, 2 * U)]:
        W = [[w[pos + o * fi + i] for i in range(fi)] for o in range(fo)]
        pos += fo * fi
        b = [w[pos + o] for o in range(fo)]
        pos += fo
        mats.append((W, b))
    out = np.zeros_like(S)
    for s in range(n_sym):
        td = [[sum(S[s, u, k] * np.exp(2j * np.pi * k * n / N) for k in range(N)) / math.sqrt(N)
               for n in range(N)] for u in range(U)]
        o_td = [[0j] * N for _ in range(U)]
        for n in range(N):
            a = []
            for u in range(U):
                for t in range(L4 + 1):
                    z = td[u][(n - t) % N]
                    a += [z.real, z.imag]
            for li, (W, b) in enumerate(mats):
                a = [b[o] + sum(W[o][i] * a[i] for i in range(len(a))) for o in range(len(b))]
                if li < len(mats) - 1:
                    a = [max(v, 0.0) for v in a]
            for u in range(U):
                o_td[u][n] = complex(a[2 * u], a[2 * u + 1])
        for u in range(U):
            for k in range(N):
                out[s, u, k] = sum(o_td[u][n] * np.exp(-2j * np.pi * k * n / N) for n in range(N)) / math.sqrt(N)
    return out


@pytest.mark.parametrize("U,L4,D,nh", [(2, 1, 3, 2), (1, 2, 4, 1)])
def test_fdnn_forward_brute_force(U, L4, D, nh):
    rng = np.random.default_rng(7)
    N = 8
    S = _rand_c(rng, 2, U, N)
    P = ofdm.fdnn_param_count(U, L4, D, nh)
    w = rng.standard_normal(P) * 0.7
    got, _ = ofdm.fdnn_forward(S, w, U, L4, D, nh)
    np.testing.assert_allclose(got, _brute_fdnn(S, w, U, L4, D, nh), atol=1e-10)


def _route_net(U, L4, src_u, src_t):
    """One hidden layer of 4U ReLU neurons that passes UE src_u[u]'s sample n - src_t
    to output u: hidden (ReLU(Re), ReLU(-Re), ReLU(Im), ReLU(-Im)), output differences."""
    F = 2 * U * (L4 + 1)
    D = 4 * U
    W1 = np.zeros((D, F))
    Wo = np.zeros((2 * U, D))
    for u in range(U):
        j = 2 * (src_u[u] * (L4 + 1) + src_t)
        W1[4 * u, j], W1[4 * u + 1, j] = 1.0, -1.0
        W1[4 * u + 2, j + 1], W1[4 * u + 3, j + 1] = 1.0, -1.0
        Wo[2 * u, 4 * u], Wo[2 * u, 4 * u + 1] = 1.0, -1.0
        Wo[2 * u + 1, 4 * u + 2], Wo[2 * u + 1, 4 * u + 3] = 1.0, -1.0
    return np.concatenate([W1.reshape(-1), np.zeros(D), Wo.reshape(-1), np.zeros(2 * U)]), D


@pytest.mark.parametrize("t", [0, 1, 3])
def test_fdnn_routing_network_is_a_cyclic_delay(t):
    """A network passing UE u+1's sample n - t to UE u gives that UE's subcarriers times
    exp(-j 2 pi k t / N) (cyclic delay theorem)."""
    rng = np.random.default_rng(3)
    U, L4, N = 3, 3, 16
    S = _rand_c(rng, 2, U, N)
    src = [(u + 1) % U for u in range(U)]
    w, D = _route_net(U, L4, src, t)
    got, _ = ofdm.fdnn_forward(S, w, U, L4, D, 1)
    ramp = np.exp(-2j * np.pi * np.arange(N) * t / N)
    np.testing.assert_allclose(got, S[:, src, :] * ramp, atol=1e-12)


def test_fdnn_backward_finite_differences():
    rng = np.random.default_rng(11)
    U, L4, D, nh, N = 2, 1, 4, 2, 8
    S = _rand_c(rng, 2, U, N)
    w = rng.standard_normal(ofdm.fdnn_param_count(U, L4, D, nh)) * 0.6
    c = _rand_c(rng, 2, U, N)                 # L = sum Re(conj(c) out): g_out = c

    def loss(v):
        o, _ = ofdm.fdnn_forward(S, v, U, L4, D, nh)
        return float(np.sum((np.conj(c) * o).real))

    _, cache = ofdm.fdnn_forward(S, w, U, L4, D, nh)
    g = ofdm.fdnn_backward(c, cache, U, L4)
    eps = 1e-6
    fd = np.array([(loss(w + eps * e) - loss(w - eps * e)) / (2 * eps) for e in np.eye(w.size)])
    np.testing.assert_allclose(g, fd, atol=1e-6)


def test_fdnn_param_layout_matches_generator():
    w = syn.xavier_fdnn(8, 3, 15, 1, 0)
    assert w.size == ofdm.fdnn_param_count(8, 3, 15, 1) == 15 * 64 + 15 + 16 * 15 + 16
    layers = ofdm.fdnn_unpack(w, 8, 3, 15, 1)
    assert [W.shape for W, _ in layers] == [(15, 64), (16, 15)]
    assert all(np.all(b == 0) for _, b in layers)


# ---------------------------------------------------------------------------
# channel and ZF
# ---------------------------------------------------------------------------
def test_channel_fd_is_the_dft_of_the_taps():
    h, _ = syn.mimo_channel(2, 5, 3, 4, 0.0, 1)
    H = ofdm.channel_fd(_c(h), 32)
    ref = np.fft.fft(_c(h), n=32, axis=1)             # sum_t H_t exp(-j 2 pi k t / N)
    np.testing.assert_allclose(H, ref, atol=1e-12)
    Hb = ofdm.channel_fd(_c(h), 32, [3, 30])
    np.testing.assert_allclose(Hb, ref[:, [3, 30]], atol=1e-12)


def test_channel_statistics():
    h, he = syn.mimo_channel(400, 10, 4, 8, 0.25, 2)
    H, E = _c(h), _c(he)
    np.testing.assert_allclose(np.mean(np.abs(H) ** 2), 0.1, rtol=0.03)
    # estimate = sqrt(.75) H + sqrt(.25) Err, Err ~ CN(0, 1)
    np.testing.assert_allclose(np.mean(np.abs(E - math.sqrt(0.75) * H) ** 2), 0.25, rtol=0.03)


def test_zf_inverts_the_estimated_channel_and_meets_the_power():
    _, he = syn.mimo_channel(2, 4, 3, 8, 0.0, 4)
    N, n_d, PT = 32, 12, 2.5
    Pt, alpha = ofdm.zf_precoder(_c(he), N, n_d, PT)
    H = ofdm.channel_fd(_c(he), N)
    I = np.eye(3)
    np.testing.assert_allclose(H @ Pt, np.broadcast_to(I, H.shape[:2] + (3, 3)), atol=1e-10)
    # Pt = H^H (H H^H)^-1 is the minimum-norm right inverse: Pt = pinv(H)
    np.testing.assert_allclose(Pt, np.linalg.pinv(H), atol=1e-10)
    # mean over data subcarriers of E||alpha Pt s||^2 with unit-energy symbols = P_T
    db = ofdm.data_bins(N, n_d)
    tr = np.sum(np.abs(Pt[:, db]) ** 2, axis=(-1, -2))
    np.testing.assert_allclose(alpha ** 2 * tr.mean(axis=1), PT, rtol=1e-12)


def test_precode_bins_and_channel_mapping():
    rng = np.random.default_rng(9)
    N, n_d, U, B = 16, 6, 2, 3
    _, he = syn.mimo_channel(2, 3, U, B, 0.0, 6)
    Pt, alpha = ofdm.zf_precoder(_c(he), N, n_d, 1.0)
    S = _rand_c(rng, 4, U, N)
    x = ofdm.precode(S, Pt, alpha, n_d, False, sym_per_ch=2)
    db = ofdm.data_bins(N, n_d)
    guard = np.setdiff1d(np.arange(N), db)
    assert np.all(x[:, :, guard] == 0)
    for i in range(4):
        c = i // 2
        for k in db:
            np.testing.assert_allclose(x[i, :, k], alpha[c] * Pt[c, k] @ S[i, :, k], atol=1e-12)
    xa = ofdm.precode(S, Pt, alpha, n_d, True, sym_per_ch=2)
    np.testing.assert_allclose(xa[:, :, db], x[:, :, db], atol=0)
    k = guard[1]
    np.testing.assert_allclose(xa[3, :, k], alpha[1] * Pt[1, k] @ S[3, :, k], atol=1e-12)


# ---------------------------------------------------------------------------
# cyclic GMP, QAM decisions
# ---------------------------------------------------------------------------
def test_gmp_cyclic_is_the_middle_of_a_periodic_stream():
    rng = np.random.default_rng(12)
    K, M, L, N = 4, 2, 2, 20
    coef = syn.gmp_coefficients(K, M, L, 3)
    x = _rand_c(rng, N) * 0.5
    got = ofdm.gmp_cyclic(x, coef, K, M, L)
    a, b, c = dpd_pa.unpack_gmp(coef, K, M, L)
    lin = dpd_pa.gmp_forward(np.tile(x, 3), a, b, c)[N:2 * N]
    np.testing.assert_allclose(got, lin, atol=1e-12)


def test_gmp_cyclic_linear():
    x = _rand_c(np.random.default_rng(1), 2, 10)
    K, M, L = 3, 1, 1
    coef = np.zeros((syn.gmp_coeff_count(K, M, L), 2))
    coef[0] = [0.5, -0.25]
    np.testing.assert_allclose(ofdm.gmp_cyclic(x, coef, K, M, L), (0.5 - 0.25j) * x, atol=1e-15)


@pytest.mark.parametrize("qam", [4, 16, 64, 256])
def test_qam_points_and_decisions(qam):
    pts = ofdm.qam_points(qam)
    np.testing.assert_allclose(pts, syn.qam_constellation(qam), atol=1e-15)
    np.testing.assert_allclose(np.mean(np.abs(pts) ** 2), 1.0, rtol=1e-12)
    idx = np.arange(qam)
    assert np.all(ofdm.qam_decide(pts, qam) == idx)
    # any perturbation shorter than half the minimum distance keeps the decision
    dmin = np.min(np.abs(pts[1:] - pts[0]))
    rng = np.random.default_rng(qam)
    ang = rng.uniform(0, 2 * np.pi, qam)
    assert np.all(ofdm.qam_decide(pts + 0.49 * dmin * np.exp(1j * ang), qam) == idx)


def test_qam_ser_closed_form_against_monte_carlo():
    rng = np.random.default_rng(21)
    qam, snr_db, n = 16, 12.0, 200_000
    snr = 10 ** (snr_db / 10)
    pts = ofdm.qam_points(qam)
    idx = rng.integers(0, qam, n)
    r = pts[idx] + _rand_c(rng, n) * math.sqrt(1 / (2 * snr))
    ser = np.mean(ofdm.qam_decide(r, qam) != idx)
    p = ofdm.qam_ser_awgn(qam, snr)
    assert abs(ser - p) < 5 * math.sqrt(p * (1 - p) / n)
    # QPSK: two independent binary decisions, Q(sqrt(snr)) each
    q = 0.5 * math.erfc(math.sqrt(10.0) / math.sqrt(2))
    assert ofdm.qam_ser_awgn(4, 10.0) == pytest.approx(1 - (1 - q) ** 2, rel=1e-12)


# ---------------------------------------------------------------------------
# link
# ---------------------------------------------------------------------------
def _link_case(n_sym=4, U=4, B=8, N=64, n_d=48, T=4, qam=16, spc=2, seed=0):
    idx, s = syn.downlink_symbols(n_sym, U, N, n_d, qam, seed)
    h, he = syn.mimo_channel(-(-n_sym // spc), T, U, B, 0.0, seed + 1)
    return idx, _c(s), _c(h), _c(he)


def test_link_linear_pa_perfect_csi_is_transparent():
    n_sym, U, B, N, n_d, qam = 4, 4, 8, 64, 48, 16
    idx, S, H, He = _link_case(n_sym, U, B, N, n_d, qam=qam)
    Pt, alpha = ofdm.zf_precoder(He, N, n_d, 1.0)
    x = ofdm.precode(S, Pt, alpha, n_d, False, 2)
    K, M, L = 3, 1, 1
    G = 0.8 + 0.3j
    pa = np.zeros((B, syn.gmp_coeff_count(K, M, L), 2))
    pa[:, 0] = [G.real, G.imag]
    dpd = np.zeros_like(pa)
    dpd[:, 0] = [1.0, 0.0]
    noise = np.zeros((n_sym, U, N), dtype=complex)
    for d in (None, dpd):
        r, dec, errs = ofdm.link(x, H, alpha, pa, (K, M, L), G, noise, idx, qam, n_d, 2,
                                 dpd_coef=d, dpd_orders=(K, M, L))
        np.testing.assert_allclose(r, S[:, :, ofdm.data_bins(N, n_d)], atol=1e-12)
        assert np.all(dec == idx) and np.all(errs == 0)


def test_link_ser_in_awgn_matches_the_closed_form():
    """Linear PA, perfect CSI: the UE sees s + w / (alpha G), so the SER is the AWGN SER
    of QAM at SNR alpha^2 |G|^2 / N0 for every symbol of a channel realisation."""
    n_sym, U, B, N, n_d, qam, spc = 8, 4, 16, 256, 192, 16, 8
    idx, S, H, He = _link_case(n_sym, U, B, N, n_d, T=6, qam=qam, spc=spc, seed=3)
    Pt, alpha = ofdm.zf_precoder(He, N, n_d, 4.0)
    x = ofdm.precode(S, Pt, alpha, n_d, False, spc)
    K, M, L = 2, 0, 0
    G = 1.0
    pa = np.zeros((B, syn.gmp_coeff_count(K, M, L), 2))
    pa[:, 0] = [G, 0.0]
    snr = 10 ** (13.0 / 10)
    n0 = alpha[0] ** 2 / snr
    noise = _c(syn.awgn_fd(n_sym, U, N, n0, 8))
    _, _, errs = ofdm.link(x, H, alpha, pa, (K, M, L), G, noise, idx, qam, n_d, spc)
    n = n_sym * U * n_d
    p = ofdm.qam_ser_awgn(qam, snr)
    assert abs(errs.sum() / n - p) < 5 * math.sqrt(p * (1 - p) / n)
    assert errs.shape == (U,)


def test_link_nonlinear_pa_adds_distortion_and_keeps_the_decisions_valid():
    n_sym, U, B, N, n_d, qam = 2, 2, 4, 64, 32, 4
    idx, S, H, He = _link_case(n_sym, U, B, N, n_d, T=3, qam=qam, spc=1, seed=5)
    Pt, alpha = ofdm.zf_precoder(He, N, n_d, 1.0)
    x = ofdm.precode(S, Pt, alpha, n_d, False, 1)
    K, M, L = 5, 2, 1
    pa = syn.antenna_pa_coefficients(B, K, M, L, 40, scale=0.3).astype(np.float64)
    noise = np.zeros((n_sym, U, N), dtype=complex)
    r, dec, errs = ofdm.link(x, H, alpha, pa, (K, M, L), 1.0, noise, idx, qam, n_d, 1)
    err = r - S[:, :, ofdm.data_bins(N, n_d)]
    assert np.sqrt(np.mean(np.abs(err) ** 2)) > 1e-3      # the PA distorts
    assert np.all(dec == ofdm.qam_decide(r, qam))
    assert errs.sum() == np.sum(dec != idx)


# ---------------------------------------------------------------------------
# adjoints (receiver-side training through the link)
# ---------------------------------------------------------------------------
def _fd_grad(f, z, eps=1e-6):
    """Real-convention gradient dL/dRe + j dL/dIm of a real f at complex z by central
    differences."""
    g = np.zeros_like(z)
    for idx in np.ndindex(z.shape):
        for unit in (1.0, 1j):
            zp = z.copy()
            zm = z.copy()
            zp[idx] += eps * unit
            zm[idx] -= eps * unit
            d = (f(zp) - f(zm)) / (2 * eps)
            g[idx] += d * unit
    return g


def test_gmp_cyclic_backward_finite_differences_and_tiling():
    rng = np.random.default_rng(31)
    K, M, L, N = 4, 2, 2, 9
    coef = syn.gmp_coefficients(K, M, L, 7)
    x = _rand_c(rng, N) * 0.6
    w = _rand_c(rng, N)
    f = lambda v: float(np.sum((np.conj(w) * ofdm.gmp_cyclic(v, coef, K, M, L)).real))
    g = ofdm.gmp_cyclic_backward(x, w, coef, K, M, L)
    np.testing.assert_allclose(g, _fd_grad(f, x), atol=1e-6)
    # chain rule through the thrice-tiled zero-padded GMP (pinned gmp_backward)
    a, b, c = dpd_pa.unpack_gmp(coef, K, M, L)
    gy = np.concatenate([np.zeros(N), w, np.zeros(N)])
    gt = dpd_pa.gmp_backward(np.tile(x, 3), gy, a, b, c)
    np.testing.assert_allclose(g, gt[:N] + gt[N:2 * N] + gt[2 * N:], atol=1e-12)


def test_link_backward_finite_differences():
    rng = np.random.default_rng(32)
    n_sym, U, B, N, n_d, T = 2, 2, 3, 8, 4, 2
    idx, S = _link_case(n_sym, U, B, N, n_d, T, qam=4, spc=1, seed=9)[:2]
    _, _, H, He = _link_case(n_sym, U, B, N, n_d, T, qam=4, spc=1, seed=9)
    Pt, alpha = ofdm.zf_precoder(He, N, n_d, 3.0)
    x = ofdm.precode(S, Pt, alpha, n_d, True, 1) + 0.1 * _rand_c(rng, n_sym, B, N)
    K, M, L = 3, 1, 1
    pa = syn.antenna_pa_coefficients(B, K, M, L, 5, scale=0.4).astype(np.float64)
    G = 0.9 + 0.2j
    w = _rand_c(rng, n_sym, U, n_d)
    noise = np.zeros((n_sym, U, N), dtype=complex)

    def f(v):
        r, _, _ = ofdm.link(v, H, alpha, pa, (K, M, L), G, noise, idx, 4, n_d, 1)
        return float(np.sum((np.conj(w) * r).real))

    g = ofdm.link_backward(w, x, H, alpha, pa, (K, M, L), G, n_d, 1)
    np.testing.assert_allclose(g, _fd_grad(f, x), atol=1e-5)


@pytest.mark.parametrize("all_bins", [False, True])
def test_precode_backward_is_the_adjoint(all_bins):
    rng = np.random.default_rng(33)
    n_sym, U, B, N, n_d, spc = 3, 2, 4, 16, 6, 2
    _, _, _, He = _link_case(n_sym, U, B, N, n_d, 3, qam=4, spc=spc, seed=4)
    Pt, alpha = ofdm.zf_precoder(He, N, n_d, 2.0)
    s = _rand_c(rng, n_sym, U, N)
    gx = _rand_c(rng, n_sym, B, N)
    lhs = np.vdot(gx, ofdm.precode(s, Pt, alpha, n_d, all_bins, spc))
    rhs = np.vdot(ofdm.precode_backward(gx, Pt, alpha, n_d, all_bins, spc), s)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)
