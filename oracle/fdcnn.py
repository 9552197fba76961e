"""FP64 oracle of the FD-CNN DPD (the paper's proposed frequency-domain CNN), forward and
reverse mode, one network applied to a batch of UE symbol vectors.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path.

Passages followed (arXiv 2205.05158):
  * a UE's data-subcarrier symbol vector (N_d complex) is written into a side x side
    matrix, side = ceil(sqrt(N_d)), in contiguous order with zero padding ... Sec. IV-A
  * its real and imaginary parts are 2 L_U real planes, convolved by N^Conv kernels of
    size K_C (stride 1 here), zero padding keeping the plane size ............ Sec. IV-A, Sec. V-A
  * an element-wise activation (ReLU), flattening, and a linear fully connected output
    layer of 2 N_d neurons: the real and imaginary parts of the predistorted symbol
    vector ...................................................................... Sec. IV-A, Sec. V-A
Readings where the paper is silent: L_U = 1 (the paper's setting; the planes are the
UE's own Re and Im); each kernel spans all input planes (a standard multi-channel
convolution, cross-correlation orientation) and has a bias; the output layer has a
bias; contiguous order = row-major (subcarrier n at row n // side, column n % side);
the flattened vector is plane-major (kernel o, row i, column j at o side^2 + i side + j);
output neuron n < N_d is Re of symbol n, N_d + n its Im.
Parameter vector (float, this order): conv weights [N^Conv][2][K_C][K_C], conv biases
[N^Conv], output weights [2 N_d][N^Conv side^2], output biases [2 N_d].
"""
from __future__ import annotations

import numpy as np


def param_count(n_d: int, side: int, n_conv: int, kc: int) -> int:
    F = n_conv * side * side
    return n_conv * 2 * kc * kc + n_conv + 2 * n_d * F + 2 * n_d


def unpack(w, n_d: int, side: int, n_conv: int, kc: int):
    w = np.asarray(w, dtype=np.float64).reshape(-1)
    F = n_conv * side * side
    sizes = [n_conv * 2 * kc * kc, n_conv, 2 * n_d * F, 2 * n_d]
    if w.size != sum(sizes):
        raise ValueError("FD-CNN parameter count does not match the shape")
    parts, pos = [], 0
    for s in sizes:
        parts.append(w[pos:pos + s])
        pos += s
    Wc = parts[0].reshape(n_conv, 2, kc, kc)
    return Wc, parts[1], parts[2].reshape(2 * n_d, F), parts[3]


def to_planes(s: np.ndarray, side: int) -> np.ndarray:
    """complex [B][N_d] -> real [B][2][side][side] (Re, Im), zero padded."""
    B, n_d = s.shape
    g = np.zeros((B, side * side), dtype=np.complex128)
    g[:, :n_d] = s
    g = g.reshape(B, side, side)
    return np.stack([g.real, g.imag], axis=1)


def conv2d_same(x: np.ndarray, Wc: np.ndarray, bc: np.ndarray) -> np.ndarray:
    """out[b][o][i][j] = bc[o] + sum_c sum_{p,q} Wc[o][c][p][q] x[b][c][i+p-h][j+q-h], zero
    outside the plane (h = K_C // 2)."""
    B, C, S, _ = x.shape
    O, _, kc, _ = Wc.shape
    h = kc // 2
    xp = np.zeros((B, C, S + 2 * h, S + 2 * h))
    xp[:, :, h:h + S, h:h + S] = x
    out = np.zeros((B, O, S, S)) + bc[None, :, None, None]
    for p in range(kc):
        for q in range(kc):
            win = xp[:, :, p:p + S, q:q + S]                  # x[.., i+p-h, j+q-h]
            out += np.einsum("oc,bcij->boij", Wc[:, :, p, q], win)
    return out


def forward(s, w, n_d: int, side: int, n_conv: int, kc: int):
    """s: complex [B][N_d] -> (predistorted symbols complex [B][N_d], cache)."""
    s = np.asarray(s, dtype=np.complex128)
    Wc, bc, Wf, bf = unpack(w, n_d, side, n_conv, kc)
    x = to_planes(s, side)
    pre = conv2d_same(x, Wc, bc)
    h = np.maximum(pre, 0.0).reshape(s.shape[0], -1)      # plane-major flattening
    y = h @ Wf.T + bf
    out = y[:, :n_d] + 1j * y[:, n_d:]
    return out, (x, pre, h, Wc, Wf)


def backward(g_out, cache, n_d: int, side: int, n_conv: int, kc: int):
    """Parameter gradient (packed like w) for the real-convention output gradient
    g_out = dL/dRe + j dL/dIm, complex [B][N_d]."""
    x, pre, h, Wc, Wf = cache
    B = x.shape[0]
    gy = np.concatenate([g_out.real, g_out.imag], axis=1)   # dL/dy [B][2 N_d]
    dWf = gy.T @ h
    dbf = gy.sum(axis=0)
    dh = (gy @ Wf).reshape(pre.shape) * (pre > 0)            # ReLU' (0 at 0)
    hh = kc // 2
    xp = np.zeros((B, 2, side + 2 * hh, side + 2 * hh))
    xp[:, :, hh:hh + side, hh:hh + side] = x
    dWc = np.zeros_like(Wc)
    for p in range(kc):
        for q in range(kc):
            dWc[:, :, p, q] = np.einsum("boij,bcij->oc", dh, xp[:, :, p:p + side, q:q + side])
    dbc = dh.sum(axis=(0, 2, 3))
    return np.concatenate([dWc.reshape(-1), dbc, dWf.reshape(-1), dbf])


def mse_to_target(out, target):
    """L = sum |out - target|^2 / (B N_d) and its real-convention gradient."""
    n = out.size
    e = out - target
    return float(np.sum(np.abs(e) ** 2) / n), 2.0 * e / n
