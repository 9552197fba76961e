"""FP64 oracle of the TDNN-DPD -> GMP-PA cascade, its NMSE and its gradient.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path:
it reads the flat input layouts (documented in dpd_synth) with its own unpacking.

Everything is plain NumPy in float64/complex128, vectorised over samples, with no
blocking or fusion beyond the definitions written out below.

Paper passages followed (arXiv 2205.05158):
  * TD DPD slot, causal window of the last L2+1 inputs ........ Sec. II-C, eq. (8)
  * tapped delay line, real/imag split, FC layers, 2 outputs ... Sec. III-C (FD-NN core)
    (per tap the TDNN here takes I, Q, |x|, |x|^2, |x|^3 and uses tanh)
  * PA with memory, filled by the GMP ............................ Sec. II-B, eq. (7); eq. (9)
  * linear-PA target x_PA = gain * x ............................. Sec. II-B
  * training by MSE through the differentiable chain ............. Sec. V-A-2
Readings where the paper is silent: taps t = 0..T-1 (T = L4 + 1), GMP memory
l = 0..M (M = L3), zero padding outside each stream on both ends (so the lead
terms of eq. (9) look ahead inside the stream), d|u|/du := 0 at u = 0,
0^0 := 1, NMSE = sum|y - G x|^2 / sum|G x|^2, loss = linear NMSE pooled over
the streams sharing one parameter set, gradients in the real convention
g_z = dL/dRe z + j dL/dIm z.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


# ---------------------------------------------------------------------------
# unpacking of the flat layouts (own code; the layout is the library's ABI)
# ---------------------------------------------------------------------------
def complex_of(a: np.ndarray) -> np.ndarray:
    """float [..., 2] (re, im) -> complex128."""
    a = np.asarray(a, dtype=np.float64)
    return a[..., 0] + 1j * a[..., 1]


def unpack_tdnn(w, taps: int, n_hidden: int, hidden: int):
    """-> list of (W [fan_out][fan_in], b [fan_out]) in float64, input layer first."""
    w = np.asarray(w, dtype=np.float64).reshape(-1)
    dims = [5 * taps] + [hidden] * n_hidden + [2]
    layers, pos = [], 0
    for i in range(len(dims) - 1):
        fi, fo = dims[i], dims[i + 1]
        W = w[pos:pos + fi * fo].reshape(fo, fi)
        pos += fi * fo
        b = w[pos:pos + fo]
        pos += fo
        layers.append((W, b))
    if pos != w.size:
        raise ValueError(f"TDNN weight vector has {w.size} floats, layout needs {pos}")
    return layers


def pack_tdnn(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


def unpack_gmp(coef, K: int, M: int, L: int):
    """-> a [K][M+1], b [K-1][M+1][L], c [K-1][M+1][L] (complex128); b/c index k-1, g-1."""
    z = complex_of(np.asarray(coef).reshape(-1, 2))
    na = K * (M + 1)
    nb = (K - 1) * (M + 1) * L
    if z.size != na + 2 * nb:
        raise ValueError("GMP coefficient count does not match (K, M, L)")
    a = z[:na].reshape(K, M + 1)
    b = z[na:na + nb].reshape(K - 1, M + 1, L)
    c = z[na + nb:].reshape(K - 1, M + 1, L)
    return a, b, c


# ---------------------------------------------------------------------------
# shifts with zero padding (stream edges)
# ---------------------------------------------------------------------------
def delay(v: np.ndarray, d: int) -> np.ndarray:
    """D(v, d)[n] = v[n - d], zero where n - d falls outside [0, len(v)).
    d < 0 looks ahead."""
    n = v.size
    out = np.zeros_like(v)
    if d >= 0:
        if d < n:
            out[d:] = v[:n - d]
    else:
        e = -d
        if e < n:
            out[:n - e] = v[e:]
    return out


def advance(v: np.ndarray, d: int) -> np.ndarray:
    """Adjoint of delay: A(v, d)[m] = v[m + d] (zero outside)."""
    return delay(v, -d)


# ---------------------------------------------------------------------------
# TDNN DPD (eq. (8) slot; Sec. III-C network core)
# ---------------------------------------------------------------------------
def features(x: np.ndarray, taps: int) -> np.ndarray:
    """Per sample n and tap t = 0..T-1 with z = x[n-t] (zero before the stream):
    (Re z, Im z, |z|, |z|^2, |z|^3) at columns 5t .. 5t+4."""
    cols = []
    for t in range(taps):
        z = delay(x, t)
        m = np.abs(z)
        cols += [z.real, z.imag, m, m * m, m * m * m]
    return np.stack(cols, axis=1)


def tdnn_forward(x: np.ndarray, layers, residual: bool = False):
    """u[n] = o0 + j o1 with o = W_o h_nl + b_o, h_i = tanh(W_i h_{i-1} + b_i), h_0 = features.
    Returns (u, [h_0, h_1, ..., h_nl])."""
    taps = layers[0][0].shape[1] // 5
    h = features(x, taps)
    hs = [h]
    for W, b in layers[:-1]:
        h = np.tanh(h @ W.T + b)
        hs.append(h)
    Wo, bo = layers[-1]
    o = h @ Wo.T + bo
    u = o[:, 0] + 1j * o[:, 1]
    if residual:
        u = u + x
    return u, hs


def tdnn_backward(hs, layers, g_u: np.ndarray):
    """Reverse mode through the TDNN for the real-convention gradient g_u.
    Returns the list of (dW, db) in the same order as `layers`."""
    delta = np.stack([g_u.real, g_u.imag], axis=1)          # d L / d o
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        h_in = hs[i]
        grads[i] = (delta.T @ h_in, delta.sum(axis=0))
        if i > 0:
            delta = (delta @ W) * (1.0 - h_in * h_in)          # tanh' = 1 - tanh^2
    return grads


# ---------------------------------------------------------------------------
# GMP PA (eq. (9)); (K, M, L) here are the paper's (K, L3, G)
# ---------------------------------------------------------------------------
def gmp_terms(K: int, M: int, L: int):
    """Every monomial of eq. (9) as (family, k, l, g, lag d) where the term is
    coef * u[n-l] * |u[n-d]|^k:  a: d = l;  b: d = l + g;  c: d = l - g."""
    out = []
    for k in range(K):
        for l in range(M + 1):
            out.append(("a", k, l, 0, l))
    for k in range(1, K):
        for l in range(M + 1):
            for g in range(1, L + 1):
                out.append(("b", k, l, g, l + g))
                out.append(("c", k, l, g, l - g))
    return out


def _coef(a, b, c, fam, k, l, g):
    if fam == "a":
        return a[k, l]
    if fam == "b":
        return b[k - 1, l, g - 1]
    return c[k - 1, l, g - 1]


def gmp_forward(u: np.ndarray, a, b, c) -> np.ndarray:
    """y[n] = sum over the monomials of eq. (9), zero-padded stream edges."""
    K, M1 = a.shape
    L = b.shape[2] if b.size else 0
    r = np.abs(u)
    y = np.zeros_like(u)
    for fam, k, l, g, d in gmp_terms(K, M1 - 1, L):
        y += _coef(a, b, c, fam, k, l, g) * delay(u, l) * delay(r, d) ** k
    return y


def _unit(u: np.ndarray) -> np.ndarray:
    """u / |u| with the value 0 at u = 0 (subgradient choice for d|u|/du)."""
    r = np.abs(u)
    out = np.zeros_like(u)
    nz = r > 0
    out[nz] = u[nz] / r[nz]
    return out


def gmp_backward(u: np.ndarray, g_y: np.ndarray, a, b, c) -> np.ndarray:
    """Real-convention gradient of a real loss w.r.t. u, given g_y.

    For a monomial y[n] += coef u[p] r[q]^k with p = n - l, q = n - d:
      g_u[p] += conj(coef r[q]^k) g_y[n]
      g_u[q] += k r[q]^(k-2) Re(conj(g_y[n]) coef u[p]) u[q]      (k >= 1)
    """
    K, M1 = a.shape
    L = b.shape[2] if b.size else 0
    r = np.abs(u)
    unit = _unit(u)
    g_u = np.zeros_like(u)
    for fam, k, l, g, d in gmp_terms(K, M1 - 1, L):
        cf = _coef(a, b, c, fam, k, l, g)
        rq = delay(r, d)
        g_u += advance(np.conj(cf) * rq ** k * g_y, l)
        if k >= 1:
            s = k * np.real(np.conj(g_y) * cf * delay(u, l))      # indexed by n
            if k == 1:
                g_u += advance(s, d) * unit
            else:
                g_u += advance(s, d) * r ** (k - 2) * u
    return g_u


# ---------------------------------------------------------------------------
# NMSE against the linear-gain target (Sec. II-B)
# ---------------------------------------------------------------------------
def nmse_parts(y: np.ndarray, x: np.ndarray, G: complex = 1.0):
    """(E, R) = (sum |y - G x|^2, sum |G x|^2)."""
    t = G * x
    e = y - t
    return float(np.sum(e.real ** 2 + e.imag ** 2)), float(np.sum(t.real ** 2 + t.imag ** 2))


def db10(v: float) -> float:
    return float(10.0 * np.log10(v)) if v > 0 else float("-inf")


# ---------------------------------------------------------------------------
# whole cascade over independent streams
# ---------------------------------------------------------------------------
@dataclass
class Model:
    taps: int
    n_hidden: int
    hidden: int
    K: int
    M: int
    L: int
    residual: bool = False


@dataclass
class CascadeResult:
    u: np.ndarray               # complex128 [n_total]
    y: np.ndarray               # complex128 [n_total]
    E: np.ndarray               # [S]
    R: np.ndarray               # [S]
    loss: np.ndarray            # [n_param_sets] pooled linear NMSE
    dw: np.ndarray | None       # [n_param_sets][P] (packed like w)


def _param_sets(w, coef, S: int, per_stream: bool):
    w = np.asarray(w, dtype=np.float64)
    coef = np.asarray(coef, dtype=np.float64)
    if per_stream:
        return [w.reshape(S, -1)[s] for s in range(S)], [coef.reshape(S, -1, 2)[s] for s in range(S)]
    return [w.reshape(-1)], [coef.reshape(-1, 2)]


def cascade(x_il, offsets, w, coef, model: Model, G: complex = 1.0,
            per_stream: bool = False, grad: bool = True) -> CascadeResult:
    """Forward (u, y), per-stream (E, R), pooled loss per parameter set and its gradient.

    x_il: float [n_total][2]; offsets: int [S+1]; streams are independent and
    zero-padded at both ends.  Stream s uses parameter set s if per_stream, else 0.
    """
    x = complex_of(x_il)
    offsets = np.asarray(offsets, dtype=np.int64)
    S = offsets.size - 1
    ws, cs = _param_sets(w, coef, S, per_stream)
    n_sets = len(ws)
    u_all = np.zeros_like(x)
    y_all = np.zeros_like(x)
    E = np.zeros(S)
    R = np.zeros(S)
    cache = []
    for s in range(S):
        lo, hi = offsets[s], offsets[s + 1]
        p = s if per_stream else 0
        layers = unpack_tdnn(ws[p], model.taps, model.n_hidden, model.hidden)
        a, b, c = unpack_gmp(cs[p], model.K, model.M, model.L)
        xs = x[lo:hi]
        u, hs = tdnn_forward(xs, layers, model.residual)
        y = gmp_forward(u, a, b, c)
        u_all[lo:hi] = u
        y_all[lo:hi] = y
        E[s], R[s] = nmse_parts(y, xs, G)
        cache.append((xs, u, y, hs, layers, (a, b, c), p))
    Rset = np.zeros(n_sets)
    Eset = np.zeros(n_sets)
    for s in range(S):
        p = cache[s][6]
        Rset[p] += R[s]
        Eset[p] += E[s]
    loss = Eset / Rset
    dw = None
    if grad:
        dw = np.zeros((n_sets, ws[0].size))
        for s in range(S):
            xs, u, y, hs, layers, (a, b, c), p = cache[s]
            g_y = 2.0 * (y - G * xs) / Rset[p]
            g_u = gmp_backward(u, g_y, a, b, c)
            grads = tdnn_backward(hs, layers, g_u)
            dw[p] += pack_tdnn(grads)
    return CascadeResult(u_all, y_all, E, R, loss, dw)


def cascade_at(x_stream: np.ndarray, idx, w, coef, model: Model):
    """u and y of one stream at the sample indices `idx`, each computed from only the
    window of inputs it depends on (x on [n - M - L - T + 1, n + L], zero outside the
    stream).  Used to check single outputs of very long streams."""
    x = complex_of(x_stream) if np.asarray(x_stream).ndim == 2 else np.asarray(x_stream)
    layers = unpack_tdnn(np.asarray(w, dtype=np.float64), model.taps, model.n_hidden, model.hidden)
    a, b, c = unpack_gmp(coef, model.K, model.M, model.L)
    back = model.M + model.L + model.taps - 1
    ahead = model.L
    N = x.size
    us, ys = [], []
    for n in np.asarray(idx).reshape(-1):
        lo = n - back
        hi = n + ahead + 1
        win = np.zeros(hi - lo, dtype=np.complex128)
        a0, a1 = max(lo, 0), min(hi, N)
        win[a0 - lo:a1 - lo] = x[a0:a1]
        # u on the window, but u itself is zero outside [0, N): the TDNN is evaluated
        # at every window position and then masked to the stream.
        u_win, _ = tdnn_forward(win, layers, model.residual)
        pos = np.arange(lo, hi)
        u_win[(pos < 0) | (pos >= N)] = 0.0
        # the window's own left edge stands in for earlier samples of x: valid because
        # u at positions >= n - M - L only looks back T - 1 samples, all inside the window
        y_win = gmp_forward(u_win, a, b, c)
        k = n - lo
        us.append(u_win[k])
        ys.append(y_win[k])
    return np.array(us), np.array(ys)
