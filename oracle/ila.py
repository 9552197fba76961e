"""FP64 oracle of the TD-GMP benchmark DPD identified by indirect learning (ILA) with
least squares.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path.

Passages followed (arXiv 2205.05158):
  * the per-antenna GMP DPD, the same monomials as eq. (9) with the DPD input in
    place of the PA input, coefficients found by mean-square-error estimation
    ......................................................... Sec. III-B, eq. (9)
  * indirect learning: a post-distorter is fitted by least squares at the output of
    each PA (PA output in, PA input as the target) and copied in front of the PA
    ......................................................... Sec. V-A-2
Readings: the post-distorter sees z = y / G (the PA output divided by the linear
target gain, so that a perfect post-inverse of a linear PA is the identity); the least
squares problem min_c sum |t - Phi(z) c|^2 is solved through its normal equations
(Phi^H Phi + lambda I) c = Phi^H t with an optional ridge lambda = ridge * tr(Phi^H Phi) / J
(ridge = 0 is plain least squares); streams are independent and zero-padded at both
ends, and streams sharing a parameter set pool their normal equations.  Column j of Phi
is the monomial that coefficient j multiplies, in the flat coefficient order of the
library (a [K][M+1], then b [K-1][M+1][L], then c [K-1][M+1][L]).
"""
from __future__ import annotations

import numpy as np

from .dpd_pa import complex_of, delay, gmp_forward, nmse_parts, unpack_gmp


def basis_matrix(z: np.ndarray, K: int, M: int, L: int) -> np.ndarray:
    """Phi [N][J] (complex128): column j = z[n-l] |z[n-q]|^k of coefficient j."""
    r = np.abs(z)
    cols = []
    for k in range(K):
        for l in range(M + 1):
            cols.append(delay(z, l) * delay(r, l) ** k)
    for sign in (+1, -1):                 # b: lag q = l + g; c: lead q = l - g
        for k in range(1, K):
            for l in range(M + 1):
                for g in range(1, L + 1):
                    cols.append(delay(z, l) * delay(r, l + sign * g) ** k)
    return np.stack(cols, axis=1)


def normal_equations(z_streams, t_streams, K: int, M: int, L: int):
    """Pooled (Phi^H Phi, Phi^H t) over streams, each with its own zero-padded basis."""
    J = K * (M + 1) + 2 * (K - 1) * (M + 1) * L
    G = np.zeros((J, J), dtype=np.complex128)
    b = np.zeros(J, dtype=np.complex128)
    for z, t in zip(z_streams, t_streams):
        Phi = basis_matrix(z, K, M, L)
        G += Phi.conj().T @ Phi
        b += Phi.conj().T @ t
    return G, b


def normal_equations_chunked(z: np.ndarray, t: np.ndarray, K: int, M: int, L: int,
                             chunk: int = 1 << 16):
    """The same sums as normal_equations for one long stream, accumulated over chunks of
    rows (bounded memory): the rows of [c0, c1) are the basis of the stream's samples
    c0..c1-1, built from the window z[c0 - M - L, c1 + L) (zero outside the stream)."""
    J = K * (M + 1) + 2 * (K - 1) * (M + 1) * L
    N = z.size
    G = np.zeros((J, J), dtype=np.complex128)
    b = np.zeros(J, dtype=np.complex128)
    back, ahead = M + L, L
    for c0 in range(0, N, chunk):
        c1 = min(N, c0 + chunk)
        lo, hi = max(0, c0 - back), min(N, c1 + ahead)
        # the window reaches M + L samples back and L ahead of its rows, so its own zero
        # padding falls only beyond the stream ends
        Phi = basis_matrix(z[lo:hi], K, M, L)[c0 - lo:c1 - lo]
        G += Phi.conj().T @ Phi
        b += Phi.conj().T @ t[c0:c1]
    return G, b


def solve_normal(G: np.ndarray, b: np.ndarray, ridge: float = 0.0) -> np.ndarray:
    J = G.shape[0]
    A = G.copy()
    if ridge:
        A += ridge * np.trace(G).real / J * np.eye(J)
    return np.linalg.solve(A, b)


def coef_array(c: np.ndarray) -> np.ndarray:
    """complex [J] -> float64 [J][2] (the library's coefficient layout)."""
    return np.stack([c.real, c.imag], axis=-1)


def ls_fit(y_il, t_il, offsets, K: int, M: int, L: int, G: complex = 1.0,
           per_stream: bool = False, ridge: float = 0.0):
    """Post-distorter fit: z = y / G, target t.  Returns per parameter set
    (coefficients float64 [J][2], Phi^H Phi, Phi^H t)."""
    y = complex_of(y_il)
    t = complex_of(t_il)
    off = np.asarray(offsets, dtype=np.int64)
    S = off.size - 1
    groups = [[s] for s in range(S)] if per_stream else [list(range(S))]
    out = []
    for grp in groups:
        zs = [y[off[s]:off[s + 1]] / G for s in grp]
        ts = [t[off[s]:off[s + 1]] for s in grp]
        Gm, b = normal_equations(zs, ts, K, M, L)
        out.append((coef_array(solve_normal(Gm, b, ridge)), Gm, b))
    return out


def gmp_apply(x_il, offsets, coef, K: int, M: int, L: int, per_stream: bool = False) -> np.ndarray:
    """GMP of eq. (9) over independent streams (coefficient set s or 0 per stream)."""
    x = complex_of(x_il)
    off = np.asarray(offsets, dtype=np.int64)
    S = off.size - 1
    cf = np.asarray(coef, dtype=np.float64).reshape(S if per_stream else 1, -1, 2)
    out = np.zeros_like(x)
    for s in range(S):
        a, b, c = unpack_gmp(cf[s if per_stream else 0], K, M, L)
        out[off[s]:off[s + 1]] = gmp_forward(x[off[s]:off[s + 1]], a, b, c)
    return out


def ila(x_il, offsets, pa_coef, pa_orders, dpd_orders, iters: int, G: complex = 1.0,
        per_stream: bool = False, ridge: float = 0.0):
    """Indirect learning: starting from the identity DPD (a_00 = 1), `iters` times run
    DPD -> PA, record the pooled NMSE of the PA output against G x, and refit the DPD as
    the post-inverse of the PA.  Returns (NMSE dB before each refit and after the last,
    final DPD coefficients [n_sets][J][2])."""
    Kd, Md, Ld = dpd_orders
    Kp, Mp, Lp = pa_orders
    off = np.asarray(offsets, dtype=np.int64)
    S = off.size - 1
    n_sets = S if per_stream else 1
    J = Kd * (Md + 1) + 2 * (Kd - 1) * (Md + 1) * Ld
    dpd = np.zeros((n_sets, J, 2))
    dpd[:, 0, 0] = 1.0
    x = complex_of(x_il)
    hist = []

    def run(d):
        u = gmp_apply(x_il, off, d, Kd, Md, Ld, per_stream)
        y = gmp_apply(np.stack([u.real, u.imag], -1), off, pa_coef, Kp, Mp, Lp, per_stream)
        E, R = nmse_parts(y, x, G)
        return u, y, 10.0 * np.log10(E / R) if E > 0 else float("-inf")

    for _ in range(iters):
        u, y, nm = run(dpd)
        hist.append(nm)
        fits = ls_fit(np.stack([y.real, y.imag], -1), np.stack([u.real, u.imag], -1), off,
                      Kd, Md, Ld, G=G, per_stream=per_stream, ridge=ridge)
        dpd = np.stack([f[0] for f in fits])
    hist.append(run(dpd)[2])
    return np.array(hist), dpd
