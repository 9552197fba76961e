"""Seeded synthetic inputs for the DPD + PA cascade.

This module is shared by the FP64 oracle, the tests and the benchmark. It only
draws and lays out inputs (OFDM-like baseband signals, GMP PA coefficients,
Xavier-initialised TDNN weights, stream lengths); none of the cascade's own
arithmetic (features, MLP, GMP, NMSE, gradients) lives here.

Signal model (Sec. II-A, eqs. (1)-(2)): i.i.d. M-QAM symbols on the data
subcarriers, guard subcarriers empty, a unitary N-point IDFT per OFDM symbol.
The paper's measured PA coefficients are not available, so the GMP PA
coefficients (eq. (9)) are drawn from a seeded complex Gaussian instead.

Flat layouts handed to the library (and unpacked independently by the oracle):
  * complex streams: float32 [n][2] interleaved (re, im)
  * TDNN weights: float32 W1[H][5T] b1[H] (W_i[H][H] b_i[H])_{i=2..nl} Wo[2][H] bo[2]
  * GMP coefficients: float32 [J][2] complex, a[K][M+1] then b[K-1][M+1][L]
    then c[K-1][M+1][L]  (b, c indexed from k = 1)
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "qam_constellation", "ofdm_signal", "papr_db", "papr_clip", "gmp_coefficients",
    "xavier_tdnn", "stream_lengths", "Workload", "WORKLOADS", "make_workload",
    "tdnn_param_count", "gmp_coeff_count", "to_interleaved", "fdcnn_symbols", "xavier_fdcnn",
    "downlink_symbols", "mimo_channel", "awgn_fd", "xavier_fdnn", "antenna_pa_coefficients",
]


# ---------------------------------------------------------------------------
# sizes of the flat parameter layouts (pure bookkeeping)
# ---------------------------------------------------------------------------
def tdnn_param_count(taps: int, n_hidden: int, hidden: int) -> int:
    """Number of floats in the packed TDNN weight vector (5 features per tap)."""
    d_in = 5 * taps
    n = hidden * d_in + hidden
    n += (n_hidden - 1) * (hidden * hidden + hidden)
    n += 2 * hidden + 2
    return n


def gmp_coeff_count(K: int, M: int, L: int) -> int:
    """Number of complex GMP coefficients J = K(M+1) + 2(K-1)(M+1)L."""
    return K * (M + 1) + 2 * (K - 1) * (M + 1) * L


def to_interleaved(z: np.ndarray) -> np.ndarray:
    """complex -> float32 [n][2] (re, im)."""
    out = np.empty(z.shape + (2,), dtype=np.float32)
    out[..., 0] = z.real
    out[..., 1] = z.imag
    return out


# ---------------------------------------------------------------------------
# OFDM-like baseband (Sec. II-A)
# ---------------------------------------------------------------------------
def qam_constellation(order: int) -> np.ndarray:
    """Square M-QAM points (2i - sqrt(M) + 1) + j(2q - sqrt(M) + 1), unit mean energy."""
    m = int(round(math.sqrt(order)))
    if m * m != order:
        raise ValueError("square QAM only")
    lv = 2.0 * np.arange(m) - m + 1.0
    pts = (lv[:, None] + 1j * lv[None, :]).reshape(-1)
    return pts / math.sqrt(np.mean(np.abs(pts) ** 2))


def ofdm_signal(n_fft: int, n_active: int, n_symbols: int, qam: int,
                rng: np.random.Generator) -> np.ndarray:
    """Concatenated OFDM symbols, unit RMS, complex128.

    Data subcarriers are +-1..+-n_active/2 (DC and the outer band empty, i.e. the
    guard subcarriers carry nothing); each symbol is a unitary IDFT (eq. (2)).
    No cyclic prefix.
    """
    if n_active % 2 or n_active >= n_fft:
        raise ValueError("n_active must be even and < n_fft")
    pts = qam_constellation(qam)
    half = n_active // 2
    bins = np.concatenate([np.arange(1, half + 1), np.arange(n_fft - half, n_fft)])
    idx = rng.integers(0, qam, size=(n_symbols, n_active))
    X = np.zeros((n_symbols, n_fft), dtype=np.complex128)
    X[:, bins] = pts[idx]
    x = np.fft.ifft(X, axis=1) * math.sqrt(n_fft)      # unitary IDFT
    x = x.reshape(-1)
    return x / math.sqrt(np.mean(np.abs(x) ** 2))


def papr_db(x: np.ndarray) -> float:
    p = np.abs(x) ** 2
    return float(10.0 * np.log10(p.max() / p.mean()))


def papr_clip(x: np.ndarray, target_db: float = 10.0, max_iter: int = 3,
              tol_db: float = 0.1) -> np.ndarray:
    """Hard amplitude clip at target_db above RMS keeping the phase, renormalise to
    unit RMS; repeated (at most max_iter times) until the PAPR is within tol_db."""
    y = x.copy()
    for _ in range(max_iter):
        rms = math.sqrt(np.mean(np.abs(y) ** 2))
        a = rms * 10.0 ** (target_db / 20.0)
        mag = np.abs(y)
        over = mag > a
        y[over] = y[over] / mag[over] * a
        y = y / math.sqrt(np.mean(np.abs(y) ** 2))
        if abs(papr_db(y) - target_db) <= tol_db:
            break
    return y


# ---------------------------------------------------------------------------
# model parameters
# ---------------------------------------------------------------------------
def gmp_coefficients(K: int, M: int, L: int, seed: int,
                     linear: complex = 1.0 + 0.0j) -> np.ndarray:
    """Seeded GMP coefficients, packed float32 [J][2].

    a_{k,l} ~ CN(0, s^2), s = 0.5^(k+l);  b_{k,l,g}, c_{k,l,g} ~ CN(0, s^2),
    s = 0.5^(k+l+g);  a_{0,0} := `linear`.  CN(0, s^2): Re, Im ~ N(0, s^2/2).
    Drawn in the order a, b, c, each in C order, from one generator.
    """
    rng = np.random.default_rng(seed)
    k = np.arange(K)[:, None]
    l = np.arange(M + 1)[None, :]
    sa = 0.5 ** (k + l)
    a = (rng.standard_normal((K, M + 1)) + 1j * rng.standard_normal((K, M + 1))) * sa / math.sqrt(2)
    a[0, 0] = linear
    kb = np.arange(1, K)[:, None, None]
    lb = np.arange(M + 1)[None, :, None]
    gb = np.arange(1, L + 1)[None, None, :]
    sb = 0.5 ** (kb + lb + gb)
    shp = (K - 1, M + 1, L)
    b = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * sb / math.sqrt(2)
    c = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * sb / math.sqrt(2)
    flat = np.concatenate([a.reshape(-1), b.reshape(-1), c.reshape(-1)])
    assert flat.size == gmp_coeff_count(K, M, L)
    return to_interleaved(flat)


def xavier_tdnn(taps: int, n_hidden: int, hidden: int, seed: int) -> np.ndarray:
    """Glorot-uniform weights U(+-sqrt(6/(fan_in+fan_out))), zero biases, packed
    float32 in layer order W1 b1 ... Wo bo, from one generator."""
    rng = np.random.default_rng(seed)
    dims = [5 * taps] + [hidden] * n_hidden + [2]
    parts = []
    for i in range(len(dims) - 1):
        fi, fo = dims[i], dims[i + 1]
        lim = math.sqrt(6.0 / (fi + fo))
        parts.append(rng.uniform(-lim, lim, size=(fo, fi)).reshape(-1))
        parts.append(np.zeros(fo))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == tdnn_param_count(taps, n_hidden, hidden)
    return w


def fdcnn_symbols(n_items: int, n_d: int, qam: int, seed: int) -> np.ndarray:
    """n_items UE symbol vectors of n_d i.i.d. QAM symbols at unit mean energy, float32
    [n_items][n_d][2] (the frequency-domain input of the FD-CNN)."""
    rng = np.random.default_rng(seed)
    pts = qam_constellation(qam)
    idx = rng.integers(0, qam, size=(n_items, n_d))
    return to_interleaved(pts[idx]).astype(np.float32)


def xavier_fdcnn(n_d: int, side: int, n_conv: int, kc: int, seed: int) -> np.ndarray:
    """Glorot-uniform FD-CNN parameters (conv fan-in 2 kc^2, fan-out n_conv kc^2; output
    layer fan-in n_conv side^2, fan-out 2 n_d), zero biases, packed float32 as the
    library's layout: conv weights, conv biases, output weights, output biases."""
    rng = np.random.default_rng(seed)
    F = n_conv * side * side
    lc = math.sqrt(6.0 / (2 * kc * kc + n_conv * kc * kc))
    lf = math.sqrt(6.0 / (F + 2 * n_d))
    w = np.concatenate([rng.uniform(-lc, lc, n_conv * 2 * kc * kc), np.zeros(n_conv),
                        rng.uniform(-lf, lf, 2 * n_d * F), np.zeros(2 * n_d)])
    return w.astype(np.float32)


# ---------------------------------------------------------------------------
# multi-user downlink (Sec. II-A): UE symbols, channels, noise, FD-NN weights
# ---------------------------------------------------------------------------
def downlink_symbols(n_sym: int, users: int, n_fft: int, n_d: int, qam: int, seed: int):
    """QAM indices int32 [n_sym][users][n_d] (point i_re sqrt(M) + i_im of
    qam_constellation) and the UE symbol vectors on the subcarriers, float32
    [n_sym][users][n_fft][2]: data symbol d on subcarrier 1 + d for d < n_d/2, else
    n_fft - n_d + d (DC and the outer band stay empty)."""
    if n_d % 2 or n_d >= n_fft:
        raise ValueError("n_d must be even and < n_fft")
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, qam, size=(n_sym, users, n_d)).astype(np.int32)
    h = n_d // 2
    bins = np.concatenate([np.arange(1, h + 1), np.arange(n_fft - h, n_fft)])
    S = np.zeros((n_sym, users, n_fft), dtype=np.complex128)
    S[:, :, bins] = qam_constellation(qam)[idx]
    return idx, to_interleaved(S).astype(np.float32)


def mimo_channel(n_ch: int, taps: int, users: int, antennas: int, eta: float, seed: int):
    """(true, estimated) tap matrices, float32 [n_ch][taps][users][antennas][2]: entries of
    the true taps ~ CN(0, 1/taps), estimate sqrt(1 - eta) H + sqrt(eta) H_err with
    H_err ~ CN(0, 1)."""
    rng = np.random.default_rng(seed)
    shp = (n_ch, taps, users, antennas)
    H = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) / math.sqrt(2.0 * taps)
    E = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) / math.sqrt(2.0)
    He = math.sqrt(1.0 - eta) * H + math.sqrt(eta) * E
    return to_interleaved(H).astype(np.float32), to_interleaved(He).astype(np.float32)


def awgn_fd(n_sym: int, users: int, n_fft: int, n0: float, seed: int) -> np.ndarray:
    """Frequency-domain receiver noise CN(0, n0) per UE and subcarrier, float32
    [n_sym][users][n_fft][2]."""
    rng = np.random.default_rng(seed)
    shp = (n_sym, users, n_fft, 2)
    return (rng.standard_normal(shp) * math.sqrt(n0 / 2.0)).astype(np.float32)


def xavier_fdnn(users: int, memory: int, hidden: int, n_hidden: int, seed: int) -> np.ndarray:
    """Glorot-uniform FD-NN weights, zero biases, packed float32 W1[D][2U(L+1)] b1[D]
    (W_i[D][D] b_i[D]) Wo[2U][D] bo[2U]."""
    rng = np.random.default_rng(seed)
    dims = [2 * users * (memory + 1)] + [hidden] * n_hidden + [2 * users]
    parts = []
    for fi, fo in zip(dims[:-1], dims[1:]):
        lim = math.sqrt(6.0 / (fi + fo))
        parts += [rng.uniform(-lim, lim, fo * fi), np.zeros(fo)]
    return np.concatenate(parts).astype(np.float32)


def antenna_pa_coefficients(antennas: int, K: int, M: int, L: int, seed: int,
                            scale: float = 1.0) -> np.ndarray:
    """One GMP coefficient set per antenna (gmp_coefficients with seeds seed + b), every
    coefficient but a_00 = 1 multiplied by `scale`: float32 [antennas][J][2]."""
    sets = []
    for b in range(antennas):
        c = gmp_coefficients(K, M, L, seed + b).astype(np.float64)
        c[1:] *= scale
        sets.append(c)
    return np.stack(sets).astype(np.float32)


def stream_lengths(n_streams: int, lo_log2: float = 14.0, hi_log2: float = 20.0,
                   seed: int = 100) -> np.ndarray:
    """Log-uniform stream lengths round(2^U(lo, hi))."""
    rng = np.random.default_rng(seed)
    return np.round(2.0 ** rng.uniform(lo_log2, hi_log2, size=n_streams)).astype(np.int64)


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    # signal
    n_fft: int
    n_active: int
    qam: int
    n_symbols: int                 # per stream (before truncation)
    papr_target_db: float | None
    # model
    taps: int
    n_hidden: int
    hidden: int
    K: int
    M: int
    L: int
    precision: str                 # "fp32" or "bf16"
    # batching
    n_streams: int = 1             # independent zero-padded streams
    frame_len: int | None = None   # equal-length frames sharing one parameter set
    per_stream_params: bool = False
    signal_seed: int = 0
    tdnn_seed: int = 1
    gmp_seed: int = 2
    description: str = ""


WORKLOADS = {
    # 8 OFDM symbols, 2048-pt IFFT, 1200 active subcarriers, 64-QAM -> 16384 samples
    "parity_16k": Workload("parity_16k", 2048, 1200, 64, 8, None, 4, 2, 20, 5, 3, 2, "fp32",
                           description="16384 samples, TDNN 4 taps 20-20, GMP K5 M3 L2"),
    # 1024 symbols, 4096-pt IFFT, 1024 active (4x oversampled) -> 2^22 samples
    "fwd_4m": Workload("fwd_4m", 4096, 1024, 64, 1024, None, 10, 3, 64, 7, 5, 3, "fp32",
                       description="2^22 samples, TDNN 10 taps 64x3, GMP K7 M5 L3, forward + ACPR"),
    # 256 symbols -> 2^20 samples as 8 frames of 131072 sharing one parameter set
    "train_1m_8f": Workload("train_1m_8f", 4096, 1024, 64, 256, None, 10, 3, 64, 7, 5, 3, "fp32",
                            frame_len=131072,
                            description="2^20 samples in 8 frames, FP32 forward+backward"),
    # 4096 symbols -> 2^24 samples, PAPR clipped to 10 dB, BF16 TDNN
    "bf16_16m": Workload("bf16_16m", 4096, 1024, 64, 4096, 10.0, 16, 4, 128, 9, 7, 4, "bf16",
                         description="2^24 samples, PAPR 10 dB, BF16-MFMA TDNN 16 taps 128x4, "
                                     "GMP K9 M7 L4, forward+backward"),
    # 64 streams, log-uniform lengths in [2^14, 2^20], own parameters per stream
    "batched_64s": Workload("batched_64s", 4096, 1024, 64, 256, None, 10, 3, 64, 7, 5, 3, "fp32",
                            n_streams=64, per_stream_params=True,
                            description="64 streams of uneven length, per-stream TDNN/GMP"),
}


@dataclass
class Inputs:
    workload: Workload
    x: np.ndarray                   # float32 [n_total][2]
    offsets: np.ndarray             # int64 [S+1]
    w: np.ndarray                   # float32 [P] or [S][P]
    coef: np.ndarray                # float32 [J][2] or [S][J][2]
    extra: dict = field(default_factory=dict)

    @property
    def n_total(self) -> int:
        return int(self.offsets[-1])


def make_workload(name_or_wl, n_streams: int | None = None, max_len: int | None = None) -> Inputs:
    """Build the seeded inputs of a named workload.

    `n_streams` limits a multi-stream workload to its first streams and `max_len`
    truncates every stream (both only to make bounded samples of a workload).
    """
    wl = WORKLOADS[name_or_wl] if isinstance(name_or_wl, str) else name_or_wl
    if wl.per_stream_params:
        S = wl.n_streams if n_streams is None else min(n_streams, wl.n_streams)
        lens = stream_lengths(wl.n_streams)[:S]
        xs, ws, cs = [], [], []
        for s in range(S):
            need = int(lens[s])
            n_sym = -(-need // wl.n_fft)
            sig = ofdm_signal(wl.n_fft, wl.n_active, n_sym, wl.qam,
                              np.random.default_rng(1000 + s))[:need]
            if max_len is not None:
                sig = sig[:max_len]
            xs.append(sig)
            ws.append(xavier_tdnn(wl.taps, wl.n_hidden, wl.hidden, 2000 + s))
            cs.append(gmp_coefficients(wl.K, wl.M, wl.L, 3000 + s))
        x = np.concatenate(xs)
        offsets = np.concatenate([[0], np.cumsum([len(v) for v in xs])]).astype(np.int64)
        return Inputs(wl, to_interleaved(x), offsets, np.stack(ws), np.stack(cs),
                      {"lengths": np.array([len(v) for v in xs])})
    rng = np.random.default_rng(wl.signal_seed)
    sig = ofdm_signal(wl.n_fft, wl.n_active, wl.n_symbols, wl.qam, rng)
    extra = {}
    if wl.papr_target_db is not None:
        sig = papr_clip(sig, wl.papr_target_db)
        extra["papr_db"] = papr_db(sig)
    n = sig.size
    if wl.frame_len is not None:
        nf = n // wl.frame_len
        lens = [wl.frame_len] * nf
    else:
        lens = [n]
    if max_len is not None or n_streams is not None:
        cap = lens[0] if max_len is None else max_len
        pieces = [sig[i * lens[0]:i * lens[0] + min(l, cap)] for i, l in enumerate(lens)]
        if n_streams is not None:
            pieces = pieces[:n_streams]
        sig = np.concatenate(pieces)
        lens = [len(p) for p in pieces]
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    w = xavier_tdnn(wl.taps, wl.n_hidden, wl.hidden, wl.tdnn_seed)
    coef = gmp_coefficients(wl.K, wl.M, wl.L, wl.gmp_seed)
    return Inputs(wl, to_interleaved(sig), offsets, w, coef, extra)
