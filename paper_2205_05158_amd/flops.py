"""Algorithmic operation counts (host-side accounting, no GPU).

The paper measures running complexity in FLOPs, counting every real addition,
subtraction and multiplication (Sec. III-A).  Its printed formulas:
  * GMP per sample, eq. (10); Fig. 3 plots 658 FLOPs/sample for K = 7, L3 = 3, G = 1
    where eq. (10) as printed gives 674.  The figure equals 8 FLOPs per complex
    coefficient of eq. (9) (J = 76) plus the magnitude/power overhead terms of
    eq. (10), i.e. eq. (10) without its subtracted triangle term; both forms are here.
  * FD-NN per UE per OFDM symbol, eq. (14), whose NN term is the per-sample cost of a
    tapped-delay-line network: 4U(L+1)D + 2(K_NN-1)D^2 + 4DU.
  * FD-CNN, eqs. (16)-(18); Fig. 3 plots 1,205,760, which equals the formulas with the
    squared grid size (ceil(sqrt(N_d))/K_S)^2 replaced by N_d; both forms are here.
The TDNN counts below follow the same rule (a multiply-add is 2 FLOPs) for the
network this library runs (5 features per tap, nl hidden layers of H, 2 outputs).
"""
from __future__ import annotations

import math


def gmp_coeffs(K: int, L3: int, G: int) -> int:
    """Number of complex coefficients of eq. (9)."""
    return K * (L3 + 1) + 2 * (K - 1) * (L3 + 1) * G


def gmp_flops_eq10(K: int, L3: int, G: int) -> int:
    """eq. (10) as printed."""
    return (8 * ((L3 + 1) * (K + 2 * K * G) - G * (G + 1) * (K - 1) // 2)
            + 10 + 2 * K + 2 * (K - 1) * G + 2 * K * min(G, L3))


def gmp_flops_fig3(K: int, L3: int, G: int) -> int:
    """Per-sample GMP FLOPs consistent with Fig. 3: 8 per complex coefficient plus the
    overhead terms of eq. (10)."""
    return 8 * gmp_coeffs(K, L3, G) + 10 + 2 * K + 2 * (K - 1) * G + 2 * K * min(G, L3)


def td_gmp_per_ue_symbol(N: int, B: int, U: int, K: int, L3: int, G: int, fig3=True) -> float:
    """eq. (11): per-sample GMP cost times N B / U."""
    c = gmp_flops_fig3(K, L3, G) if fig3 else gmp_flops_eq10(K, L3, G)
    return c * N * B / U


def fd_nn_per_ue_symbol(N: int, Nd: int, B: int, U: int, L: int, D: int, K_nn: int) -> float:
    """eq. (14)."""
    nn = N * (4 * U * (L + 1) * D + 2 * (K_nn - 1) * D * D + 4 * D * U)
    dft = 10 * U * N * math.log2(N)
    extra = (6 + 2) * (N - Nd) * U * B
    return (nn + dft + extra) / U


def fd_cnn_per_ue_symbol(Nd: int, L_U: int, K_C: int, K_S: int, N_conv: int, fig3=True) -> float:
    """eqs. (16)-(18)."""
    side = math.ceil(math.sqrt(Nd))
    grid = Nd if fig3 else (side / K_S) ** 2
    conv = 2 * N_conv * L_U * (2 * K_C * K_C - 1) * grid
    fc = 8 * Nd * L_U * grid
    return conv + fc


def tdnn_flops(taps: int, n_hidden: int, hidden: int) -> dict:
    """Per-sample FLOPs of the TDNN of this library, split by the unit that runs them.
    fwd_mma: input + hidden layers (MFMA); out: the 2-output layer (vector ALU);
    bwd_mma: dW of input + hidden layers and dX of hidden layers >= 2 (MFMA);
    bwd_out: dW of the output layer and its dX (vector ALU)."""
    d_in, H = 5 * taps, hidden
    fwd = 2 * (d_in * H + (n_hidden - 1) * H * H)
    out = 2 * 2 * H
    bwd = fwd + 2 * (n_hidden - 1) * H * H
    bwd_out = 2 * (2 * 2 * H)
    return {"fwd_mma": fwd, "out": out, "bwd_mma": bwd, "bwd_out": bwd_out,
            "total": fwd + out + bwd + bwd_out}


def gmp_train_flops(K: int, M: int, L: int) -> dict:
    """Per-sample GMP FLOPs: forward per Fig. 3's reading of eq. (10); the reverse mode
    with respect to the PA input costs two forward passes (one per use of each sample:
    as the multiplied sample and inside the envelope)."""
    f = gmp_flops_fig3(K, M, L)
    return {"fwd": f, "bwd": 2 * f, "total": 3 * f}


# ---------------------------------------------------------------- executed counts
# The kernels evaluate eq. (9) in the factorised form y[n] = sum_l u[n-l] Q_l(n-l), each
# Q_l a polynomial in |u| at one position (and its neighbours for the b, c families)
# evaluated by Horner's rule: one complex-by-real fused multiply-add (4 FLOPs) per
# coefficient instead of the 8 FLOPs per complex coefficient that eq. (10) counts for the
# direct sum of products.  These counts are what the kernels execute (a multiply-add is
# 2 FLOPs), and what their vector-ALU roofline is taken against.

def gmp_q_executed(K: int, M: int, L: int) -> int:
    """FLOPs of all M + 1 polynomials Q_l at one position: the a family by Horner over
    k = 0..K-1 (4 (K - 1)), per lag g the b and c families over k = 1..K-1 (4 (K - 2)
    each) and their combination (8)."""
    per_l = 4 * (K - 1)
    if K > 1:
        per_l += L * (2 * 4 * (K - 2) + 8)
    return (M + 1) * per_l


def gmp_y_executed(M: int) -> int:
    """FLOPs of y[n] = sum_l u[n-l] Q_l(n-l): a complex product and accumulation per tap."""
    return 8 * (M + 1)


def gmp_grad_executed(K: int, M: int, L: int) -> int:
    """FLOPs of the gather-form reverse mode at one sample: conj(Q_l) g_y per tap (8),
    and per envelope term (the a family, and per lag the b and c families) the weight
    conj(g_y) u (6), its products with C_1 (4) and with the Horner sum of k C_k r^(k-2)
    (4 + 4 (K - 3)); 10 for the final combination."""
    d2 = 4 * max(K - 3, 0)
    per_l = 8
    if K > 1:
        env = 6 + 4 + d2 + 4
        per_l += env + 2 * L * env
    return (M + 1) * per_l + 10


def gmp_bwd_executed(K: int, M: int, L: int, tile: int) -> float:
    """Per sample of the TD reverse-mode GMP kernel with `tile`-sample tiles: Q on the tile
    and a halo of M + L positions each side, y, error and gradient seed (8 more FLOPs)
    on the tile plus L behind and M + L ahead, the gather-form gradient on the tile."""
    q = gmp_q_executed(K, M, L) * (tile + 2 * (M + L)) / tile
    y = (gmp_y_executed(M) + 8) * (tile + M + 2 * L) / tile
    return q + y + gmp_grad_executed(K, M, L)


def fft_nominal(n: int) -> float:
    """Per-point FLOPs of one n-point complex FFT, the radix-2 nominal 5 log2 n."""
    return 5 * math.log2(n)


def link_pa_executed(K: int, M: int, L: int, n: int) -> float:
    """Per sample of the cyclic PA kernel of the downlink (one antenna row): IDFT, Q and y
    on every sample (cyclic: no halo), DFT."""
    return gmp_q_executed(K, M, L) + gmp_y_executed(M) + 2 * fft_nominal(n)


def link_pa_bwd_executed(K: int, M: int, L: int, n: int) -> float:
    """Per sample of its reverse mode: IDFT of x and of the output gradient, Q, the
    gather-form gradient, DFT."""
    return gmp_q_executed(K, M, L) + gmp_grad_executed(K, M, L) + 3 * fft_nominal(n)
