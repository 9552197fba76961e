"""FP64 oracle of the multi-user OFDM downlink around the frequency-domain DPDs: the
FD-NN wrapper (per-UE IDFT, delay-line network over all UEs, per-UE DFT), ZF
precoding, and a link of per-antenna PAs, a frequency-selective channel, AWGN and
symbol decisions for the symbol error rate.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path.

Passages followed (arXiv 2205.05158):
  * N subcarriers, N_d of them data and the rest guard; per subcarrier the precoder maps
    the U UE symbols to B antennas, and is zero on guard subcarriers ...... Sec. II-A, eq. (1)
  * a unitary N-point IDFT per antenna gives the time-domain signal ...... Sec. II-A, eq. (2)
  * a T-tap channel; its frequency-domain matrices are the tap sums weighted by
    exp(-j 2 pi k t / N), and the received subcarrier is H_k x_k + w_k .... Sec. II-A, eqs. (3)-(5)
  * ZF precoding: alpha H_k^H (H_k H_k^H)^-1 with alpha meeting the average transmit
    power, built from the estimated channel sqrt(1-eta) H + sqrt(eta) H_err ... Sec. II-A, eq. (6)
  * a PA with memory per antenna (here the GMP of eq. (9)); optionally a per-antenna
    TD-GMP DPD in front of it ............................................ Sec. II-B/C, eqs. (7)-(9)
  * FD-NN: each UE's symbol vector to the time domain by an IDFT, delay lines of L4 + 1
    samples of all U UEs as 2 U (L4 + 1) real inputs, K^NN fully connected ReLU layers
    of D neurons, 2 U linear outputs, and a DFT per UE back to the subcarriers .. Sec. III-C
  * symbol error rate over the QAM symbols of the data subcarriers ....... Sec. V-B
  * supervised training of the frequency-domain DPDs through all simulated blocks with a
    loss at the receiver: the adjoints of precoding and of the link ........ Sec. V-A-2
Readings where the paper is silent or loose:
  * data subcarriers are +-1..+-N_d/2 (DC and the outer band are guard), as for the
    time-domain signals;
  * every delay inside an OFDM symbol is cyclic (index mod N): the frequency-domain form
    of the channel holds exactly only for a cyclic convolution, i.e. with a cyclic prefix
    longer than every memory, and the FD-NN delay lines, the DPD and the PA then read the
    same cyclic symbol;
  * the received subcarriers are the unitary DFT of the received samples (with the
    unnormalised sum the received vector would carry an extra sqrt(N) against eq. (2));
    the frequency-domain noise is then CN(0, N_0) per UE and subcarrier;
  * one alpha per channel realisation: alpha^2 times the mean over the data subcarriers
    of tr(Pt_k^H Pt_k) equals P_T (unit-energy symbols), Pt_k = H_k^H (H_k H_k^H)^-1;
    guard subcarriers use the same alpha when they are precoded (FD-NN);
  * FD-NN input order: feature 2 (u (L4+1) + t) + {0: Re, 1: Im} is UE u's sample
    n - t; output neuron 2u is Re and 2u + 1 Im of UE u; parameters
    W1[D][2U(L4+1)] b1[D] (W_i[D][D] b_i[D])_{i=2..K^NN} Wo[2U][D] bo[2U];
  * the UE scales its received sample by 1 / (alpha G), G the PA's linear gain, and
    decides the nearest point of the unit-energy square QAM, whose point i_re sqrt(M) +
    i_im is (2 i_re - sqrt(M) + 1) + j (2 i_im - sqrt(M) + 1), normalised.
"""
from __future__ import annotations

import math

import numpy as np

from .dpd_pa import unpack_gmp


# ---------------------------------------------------------------------------
# unitary DFT pair (eq. (2) and its inverse)
# ---------------------------------------------------------------------------
def dft(x: np.ndarray) -> np.ndarray:
    """X_k = N^-1/2 sum_n x_n exp(-j 2 pi k n / N) along the last axis."""
    return np.fft.fft(np.asarray(x, dtype=np.complex128), axis=-1, norm="ortho")


def idft(X: np.ndarray) -> np.ndarray:
    """x_n = N^-1/2 sum_k X_k exp(+j 2 pi k n / N) along the last axis (eq. (2))."""
    return np.fft.ifft(np.asarray(X, dtype=np.complex128), axis=-1, norm="ortho")


def data_bins(n_fft: int, n_d: int) -> np.ndarray:
    """Subcarrier indices of the data symbols, in symbol order: +1..+N_d/2 then
    N - N_d/2..N - 1 (negative frequencies)."""
    h = n_d // 2
    return np.concatenate([np.arange(1, h + 1), np.arange(n_fft - h, n_fft)])


# ---------------------------------------------------------------------------
# FD-NN (Sec. III-C)
# ---------------------------------------------------------------------------
def fdnn_param_count(users: int, memory: int, hidden: int, n_hidden: int) -> int:
    F = 2 * users * (memory + 1)
    return hidden * F + hidden + (n_hidden - 1) * (hidden * hidden + hidden) + 2 * users * hidden + 2 * users


def fdnn_unpack(w, users: int, memory: int, hidden: int, n_hidden: int):
    w = np.asarray(w, dtype=np.float64).reshape(-1)
    if w.size != fdnn_param_count(users, memory, hidden, n_hidden):
        raise ValueError("FD-NN parameter count does not match the shape")
    shapes = [(hidden, 2 * users * (memory + 1))] + [(hidden, hidden)] * (n_hidden - 1) + [(2 * users, hidden)]
    layers, pos = [], 0
    for r, c in shapes:
        W = w[pos:pos + r * c].reshape(r, c)
        pos += r * c
        layers.append((W, w[pos:pos + r]))
        pos += r
    return layers


def fdnn_features(s_td: np.ndarray, memory: int) -> np.ndarray:
    """s_td complex [n_sym][U][N] -> real [n_sym][N][2 U (L4+1)], cyclic delays."""
    n_sym, U, N = s_td.shape
    f = np.zeros((n_sym, N, 2 * U * (memory + 1)))
    for u in range(U):
        for t in range(memory + 1):
            z = np.roll(s_td[:, u, :], t, axis=-1)          # z[n] = s[(n - t) mod N]
            j = 2 * (u * (memory + 1) + t)
            f[:, :, j] = z.real
            f[:, :, j + 1] = z.imag
    return f


def fdnn_forward(s_fd, w, users: int, memory: int, hidden: int, n_hidden: int):
    """s_fd complex [n_sym][U][N] (subcarriers) -> (predistorted complex [n_sym][U][N],
    cache).  IDFT per UE, the network per time sample, DFT per UE."""
    s_fd = np.asarray(s_fd, dtype=np.complex128)
    layers = fdnn_unpack(w, users, memory, hidden, n_hidden)
    s_td = idft(s_fd)
    h = fdnn_features(s_td, memory)
    acts = [h]
    for W, b in layers[:-1]:
        h = np.maximum(h @ W.T + b, 0.0)
        acts.append(h)
    Wo, bo = layers[-1]
    o = h @ Wo.T + bo                                       # [n_sym][N][2U]
    o_td = np.transpose(o[..., 0::2] + 1j * o[..., 1::2], (0, 2, 1))
    return dft(o_td), (acts, layers)


def fdnn_backward(g_out, cache, users: int, memory: int):
    """Parameter gradient (packed like w) for the real-convention output gradient
    g_out = dL/dRe + j dL/dIm, complex [n_sym][U][N].  The adjoint of the unitary DFT is
    the unitary IDFT."""
    acts, layers = cache
    g_td = idft(g_out)                                      # [n_sym][U][N]
    g = np.zeros(acts[-1].shape[:-1] + (2 * users,))
    g[..., 0::2] = np.transpose(g_td.real, (0, 2, 1))
    g[..., 1::2] = np.transpose(g_td.imag, (0, 2, 1))
    grads = []
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        a = acts[i]
        g2 = g.reshape(-1, g.shape[-1])
        grads.append((g2.T @ a.reshape(-1, a.shape[-1]), g2.sum(axis=0)))
        if i > 0:
            g = (g @ W) * (acts[i] > 0)                     # ReLU' (0 at 0)
    grads.reverse()
    return np.concatenate([np.concatenate([dW.reshape(-1), db]) for dW, db in grads])


# ---------------------------------------------------------------------------
# channel and ZF precoding (Sec. II-A)
# ---------------------------------------------------------------------------
def channel_fd(h_taps: np.ndarray, n_fft: int, bins=None) -> np.ndarray:
    """h_taps complex [n_ch][T][U][B] -> H_k complex [n_ch][len(bins)][U][B],
    H_k = sum_t H_t exp(-j 2 pi k t / N) (all N bins by default)."""
    h_taps = np.asarray(h_taps, dtype=np.complex128)
    k = np.arange(n_fft) if bins is None else np.asarray(bins)
    T = h_taps.shape[1]
    ph = np.exp(-2j * np.pi * np.outer(k, np.arange(T)) / n_fft)     # [K][T]
    return np.einsum("kt,ctub->ckub", ph, h_taps)


def zf_precoder(h_est_taps, n_fft: int, n_d: int, p_total: float):
    """-> (Pt complex [n_ch][N][B][U] with Pt_k = H_k^H (H_k H_k^H)^-1 on every
    subcarrier, alpha float [n_ch]) so that P_k = alpha Pt_k."""
    H = channel_fd(h_est_taps, n_fft)                       # [n_ch][N][U][B]
    Hh = np.conj(np.swapaxes(H, -1, -2))                    # [n_ch][N][B][U]
    Pt = Hh @ np.linalg.inv(H @ Hh)
    db = data_bins(n_fft, n_d)
    tr = np.sum(np.abs(Pt[:, db]) ** 2, axis=(-1, -2))      # tr(Pt^H Pt) per data bin
    alpha = np.sqrt(p_total / tr.mean(axis=1))
    return Pt, alpha


def precode(s_fd, Pt, alpha, n_d: int, all_bins: bool = False, sym_per_ch: int = 1):
    """s_fd complex [n_sym][U][N] -> x complex [n_sym][B][N], x_k = alpha Pt_k s_k on the
    data subcarriers (and on the guard subcarriers too when all_bins), zero elsewhere.
    OFDM symbol i uses channel realisation i // sym_per_ch."""
    s_fd = np.asarray(s_fd, dtype=np.complex128)
    n_sym, U, N = s_fd.shape
    B = Pt.shape[2]
    x = np.zeros((n_sym, B, N), dtype=np.complex128)
    bins = np.arange(N) if all_bins else data_bins(N, n_d)
    for i in range(n_sym):
        c = i // sym_per_ch
        for k in bins:
            x[i, :, k] = alpha[c] * (Pt[c, k] @ s_fd[i, :, k])
    return x


# ---------------------------------------------------------------------------
# per-antenna GMP with cyclic delays, QAM decisions, the link
# ---------------------------------------------------------------------------
def gmp_cyclic(x: np.ndarray, coef, K: int, M: int, L: int) -> np.ndarray:
    """eq. (9) along the last axis with every delay taken mod N."""
    a, b, c = unpack_gmp(coef, K, M, L)
    r = np.abs(x)
    y = np.zeros_like(x, dtype=np.complex128)
    for l in range(M + 1):
        ul = np.roll(x, l, axis=-1)                          # x[n - l]
        for k in range(K):
            y += a[k, l] * ul * np.roll(r, l, axis=-1) ** k
        for k in range(1, K):
            for g in range(1, L + 1):
                y += b[k - 1, l, g - 1] * ul * np.roll(r, l + g, axis=-1) ** k
                y += c[k - 1, l, g - 1] * ul * np.roll(r, l - g, axis=-1) ** k
    return y


def gmp_cyclic_backward(x: np.ndarray, g_y: np.ndarray, coef, K: int, M: int, L: int) -> np.ndarray:
    """Real-convention gradient (dL/dRe + j dL/dIm) with respect to x of a real loss through
    gmp_cyclic, given g_y for its output: each monomial c x[n - l] |x[n - q]|^k of eq. (9)
    differentiated on its own, delays mod N.  The multiplied sample gives
    conj(c |x[n - q]|^k) g_y[n] at n - l; the envelope (k >= 1) gives
    k |x[n - q]|^(k-1) Re(conj(g_y[n]) c x[n - l]) x[n - q] / |x[n - q]| at n - q (0 at x = 0)."""
    a, b, c = unpack_gmp(coef, K, M, L)
    x = np.asarray(x, dtype=np.complex128)
    r = np.abs(x)
    unit = np.zeros_like(x)
    nz = r > 0
    unit[nz] = x[nz] / r[nz]
    terms = [(a[k, l], k, l, l) for l in range(M + 1) for k in range(K)]
    terms += [(b[k - 1, l, g - 1], k, l, l + g) for k in range(1, K) for l in range(M + 1) for g in range(1, L + 1)]
    terms += [(c[k - 1, l, g - 1], k, l, l - g) for k in range(1, K) for l in range(M + 1) for g in range(1, L + 1)]
    out = np.zeros_like(x)
    for cf, k, l, q in terms:
        rq = np.roll(r, q, axis=-1)                                  # |x[n - q]|
        out += np.roll(np.conj(cf) * rq ** k * g_y, -l, axis=-1)    # to index n - l
        if k >= 1:
            s = k * np.real(np.conj(g_y) * cf * np.roll(x, l, axis=-1))
            out += np.roll(s, -q, axis=-1) * r ** (k - 1) * unit    # to index n - q
    return out


def link_backward(g_r, x_fd, h_taps, alpha, pa_coef, pa_orders, G: complex, n_d: int, sym_per_ch: int = 1):
    """Adjoint of `link` (no DPD, no decisions) for the real-convention gradient g_r of a
    real loss with respect to the equalised data symbols (complex [n_sym][U][N_d]): the
    gradient with respect to the precoded antenna subcarriers x_fd ([n_sym][B][N]).
    Equalisation and channel are complex-linear (adjoint: the conjugate transpose), the
    unitary DFT's adjoint is the IDFT and vice versa, the PA goes through
    gmp_cyclic_backward."""
    x_fd = np.asarray(x_fd, dtype=np.complex128)
    n_sym, B, N = x_fd.shape
    K, M, L = pa_orders
    u = idft(x_fd)
    db = data_bins(N, n_d)
    H = channel_fd(h_taps, N, db)                           # [n_ch][N_d][U][B]
    g_y = np.zeros_like(x_fd)
    for i in range(n_sym):
        c = i // sym_per_ch
        g_z = np.conj(1.0 / (alpha[c] * G)) * np.asarray(g_r)[i]       # [U][N_d]
        g_y[i][:, db] = np.einsum("kub,uk->bk", np.conj(H[c]), g_z)
    g_y_td = idft(g_y)
    g_u = np.stack([gmp_cyclic_backward(u[:, b], g_y_td[:, b], pa_coef[b], K, M, L) for b in range(B)], axis=1)
    return dft(g_u)


def precode_backward(g_x, Pt, alpha, n_d: int, all_bins: bool = False, sym_per_ch: int = 1):
    """Adjoint of `precode`: g_s[i][:, k] = alpha Pt_k^H g_x[i][:, k] on the precoded
    subcarriers, 0 elsewhere ([n_sym][B][N] -> [n_sym][U][N])."""
    g_x = np.asarray(g_x, dtype=np.complex128)
    n_sym, B, N = g_x.shape
    U = Pt.shape[3]
    g_s = np.zeros((n_sym, U, N), dtype=np.complex128)
    bins = np.arange(N) if all_bins else data_bins(N, n_d)
    for i in range(n_sym):
        c = i // sym_per_ch
        for k in bins:
            g_s[i, :, k] = alpha[c] * (np.conj(Pt[c, k]).T @ g_x[i, :, k])
    return g_s


def qam_points(qam: int) -> np.ndarray:
    m = int(round(math.sqrt(qam)))
    lv = 2.0 * np.arange(m) - m + 1.0
    pts = (lv[:, None] + 1j * lv[None, :]).reshape(-1)
    return pts / math.sqrt(np.mean(np.abs(pts) ** 2))


def qam_decide(r: np.ndarray, qam: int) -> np.ndarray:
    """Index of the nearest constellation point (exhaustive search)."""
    pts = qam_points(qam)
    r = np.asarray(r)
    d = np.abs(r.reshape(-1, 1) - pts[None, :]) ** 2
    return np.argmin(d, axis=1).reshape(r.shape)


def link(x_fd, h_taps, alpha, pa_coef, pa_orders, G: complex, noise_fd, tx_idx, qam: int,
         n_d: int, sym_per_ch: int = 1, dpd_coef=None, dpd_orders=None):
    """Precoded x_fd complex [n_sym][B][N] through IDFT, the optional per-antenna TD-GMP
    DPD (coefficients [B][Jd][2]), the per-antenna PA (coefficients [B][J][2]), DFT, the
    true channel and the FD noise noise_fd complex [n_sym][U][N].  Returns (equalised
    data symbols complex [n_sym][U][N_d] = y_k / (alpha G), decisions int [n_sym][U][N_d],
    symbol errors per UE int [U]) against tx_idx int [n_sym][U][N_d]."""
    x_fd = np.asarray(x_fd, dtype=np.complex128)
    n_sym, B, N = x_fd.shape
    u = idft(x_fd)
    if dpd_coef is not None:
        Kd, Md, Ld = dpd_orders
        u = np.stack([gmp_cyclic(u[:, b], dpd_coef[b], Kd, Md, Ld) for b in range(B)], axis=1)
    K, M, L = pa_orders
    y_td = np.stack([gmp_cyclic(u[:, b], pa_coef[b], K, M, L) for b in range(B)], axis=1)
    y_fd = dft(y_td)
    db = data_bins(N, n_d)
    H = channel_fd(h_taps, N, db)                           # [n_ch][N_d][U][B]
    U = H.shape[2]
    r = np.zeros((n_sym, U, n_d), dtype=np.complex128)
    for i in range(n_sym):
        c = i // sym_per_ch
        yk = np.einsum("kub,bk->uk", H[c], y_fd[i][:, db]) + np.asarray(noise_fd)[i][:, db]
        r[i] = yk / (alpha[c] * G)
    dec = qam_decide(r, qam)
    errs = np.sum(dec != np.asarray(tx_idx), axis=(0, 2))
    return r, dec, errs


def qam_ser_awgn(qam: int, snr: float) -> float:
    """Closed-form symbol error probability of square M-QAM in AWGN at symbol SNR snr
    (textbook: 1 - (1 - 2 (1 - 1/sqrt(M)) Q(sqrt(3 snr / (M - 1))))^2)."""
    m = math.sqrt(qam)
    q = 0.5 * math.erfc(math.sqrt(3.0 * snr / (qam - 1)) / math.sqrt(2.0))
    p = 2.0 * (1.0 - 1.0 / m) * q
    return 1.0 - (1.0 - p) ** 2
