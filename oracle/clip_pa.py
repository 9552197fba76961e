"""FP64 oracle of the ideal linear-clipping PA and of the cascade TDNN-DPD ->
clipping PA -> NMSE with its gradient.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; it shares no code with the HIP path.

Paper passage followed (arXiv 2205.05158): the SER comparison of Sec. V-B-2 adds an
ideal linear-clipping PA as the minimum-distortion reference: linear before its
clipping region.  Reading where the paper gives no formula: unit small-signal gain
(any other linear gain is the target gain G of the NMSE), a hard envelope limit at
the clipping level A with the phase kept, no memory:
    y = u                  for |u| <= A
    y = A u / |u|          for |u| >  A.
Its reverse mode in the real convention g_z = dL/dRe z + j dL/dIm z: below the clip
g_u = g_y; beyond it y depends on the phase of u only, the Jacobian of A u/|u| being
(A/|u|)(I - v v^T) with v = u/|u|, so g_u = (A/|u|)(g_y - v Re(conj(v) g_y)).  At
|u| = A the linear branch's derivative is taken.  The DPD, the loss (linear NMSE
pooled over the streams of a parameter set) and the TDNN reverse mode are those of
dpd_pa.py.
"""
from __future__ import annotations

import numpy as np

from .dpd_pa import (CascadeResult, Model, complex_of, nmse_parts, pack_tdnn, tdnn_backward,
                     tdnn_forward, unpack_tdnn)


def clip_forward(u: np.ndarray, A: float) -> np.ndarray:
    """The clipping PA: u where |u| <= A, A u / |u| elsewhere."""
    u = np.asarray(u, dtype=np.complex128)
    r = np.abs(u)
    y = u.copy()
    over = r > A
    y[over] = A * u[over] / r[over]
    return y


def clip_backward(u: np.ndarray, g_y: np.ndarray, A: float) -> np.ndarray:
    """Real-convention gradient w.r.t. u of a real loss with gradient g_y w.r.t. y."""
    u = np.asarray(u, dtype=np.complex128)
    g_u = np.array(g_y, dtype=np.complex128)
    r = np.abs(u)
    over = r > A
    v = u[over] / r[over]
    g = g_u[over]
    g_u[over] = (A / r[over]) * (g - v * np.real(np.conj(v) * g))
    return g_u


def cascade_clip(x_il, offsets, w, model: Model, A: float, G: complex = 1.0,
                 per_stream: bool = False, grad: bool = True) -> CascadeResult:
    """Forward (u, y), per-stream (E, R), pooled loss per parameter set and its gradient
    for the DPD followed by the clipping PA.  model.K, M, L are unused."""
    x = complex_of(x_il)
    offsets = np.asarray(offsets, dtype=np.int64)
    S = offsets.size - 1
    w = np.asarray(w, dtype=np.float64)
    ws = [w.reshape(S, -1)[s] for s in range(S)] if per_stream else [w.reshape(-1)]
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
        xs = x[lo:hi]
        u, hs = tdnn_forward(xs, layers, model.residual)
        y = clip_forward(u, A)
        u_all[lo:hi] = u
        y_all[lo:hi] = y
        E[s], R[s] = nmse_parts(y, xs, G)
        cache.append((xs, u, y, hs, layers, p))
    Eset = np.zeros(n_sets)
    Rset = np.zeros(n_sets)
    for s in range(S):
        Eset[cache[s][5]] += E[s]
        Rset[cache[s][5]] += R[s]
    loss = Eset / Rset
    dw = None
    if grad:
        dw = np.zeros((n_sets, ws[0].size))
        for xs, u, y, hs, layers, p in cache:
            g_y = 2.0 * (y - G * xs) / Rset[p]
            g_u = clip_backward(u, g_y, A)
            dw[p] += pack_tdnn(tdnn_backward(hs, layers, g_u))
    return CascadeResult(u_all, y_all, E, R, loss, dw)
