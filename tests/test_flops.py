"""The FLOP accounting reproduces every value printed in Fig. 3 (Sec. V-B-1)
under the readings stated in paper_2205_05158_amd/flops.py."""
import os

import numpy as np

from paper_2205_05158_amd import flops as F

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig3_flops.txt")


def test_fig3_every_entry():
    rows = np.loadtxt(GOLD, dtype=np.int64)
    for B, g1, g4, g8, fdnn, fdcnn in rows:
        for U, ref in ((1, g1), (4, g4), (8, g8)):
            assert F.td_gmp_per_ue_symbol(4096, B, U, 7, 3, 1) == ref
        for U in (1, 4, 8):
            assert F.fd_nn_per_ue_symbol(4096, 384, B, U, 3, 15, 1) == fdnn
        assert F.fd_cnn_per_ue_symbol(384, 1, 3, 1, 2) == fdcnn


def test_printed_formulas_differ_from_fig3_as_stated():
    assert F.gmp_flops_eq10(7, 3, 1) == 674
    assert F.gmp_flops_fig3(7, 3, 1) == 658
    assert F.fd_cnn_per_ue_symbol(384, 1, 3, 1, 2, fig3=False) == 1256000


def test_fd_nn_network_term_is_tdnn_count_with_two_features():
    # eq. (14)'s NN term for U = 1, L4 = 3, D = 15, one hidden layer = 300 FLOPs/sample
    nn = 4 * 1 * 4 * 15 + 0 + 4 * 15
    assert nn == 300


def test_tdnn_counts():
    f = F.tdnn_flops(16, 4, 128)
    assert f["fwd_mma"] == 2 * (80 * 128 + 3 * 128 * 128)
    assert f["fwd_mma"] + f["out"] + f["bwd_mma"] + f["bwd_out"] == f["total"]
    assert F.gmp_coeffs(9, 7, 4) == 584


def test_executed_gmp_counts_follow_the_coefficient_count():
    """Horner evaluation costs 4 FLOPs (one complex-by-real multiply-add) per coefficient
    beyond the leading one of each polynomial: (M + 1) polynomials of the a family and
    2 L (M + 1) of the b and c families, plus 8 FLOPs per (l, g) to combine them; the
    executed count is below eq. (10)'s 8 FLOPs per coefficient."""
    for K in range(2, 10):
        for M in range(0, 8):
            for L in range(0, 5):
                J = F.gmp_coeffs(K, M, L)
                polys = (M + 1) * (1 + 2 * L)
                assert F.gmp_q_executed(K, M, L) == 4 * (J - polys) + 8 * (M + 1) * L
                assert F.gmp_q_executed(K, M, L) < F.gmp_flops_fig3(K, M, L)
    assert F.gmp_q_executed(1, 0, 0) == 0 and F.gmp_y_executed(0) == 8
    # the headline PA (9, 7, 4): about 5.4k FLOPs per sample for the whole reverse-mode
    # kernel against 3 x 4836 = 14508 counted with eq. (10)
    assert 5300 < F.gmp_bwd_executed(9, 7, 4, 256) < 5500
    assert 3 * F.gmp_flops_fig3(9, 7, 4) == 14508
    # the downlink's cyclic PA kernels (no halo): Q and y (forward) or the gather-form
    # gradient (reverse) on every sample, plus two or three n-point transforms at 5 log2 n
    for K, M, L in ((7, 3, 1), (9, 7, 4), (5, 3, 2)):
        q = F.gmp_q_executed(K, M, L)
        assert F.link_pa_executed(K, M, L, 4096) == q + F.gmp_y_executed(M) + 2 * 5 * 12
        assert F.link_pa_bwd_executed(K, M, L, 4096) == q + F.gmp_grad_executed(K, M, L) + 3 * 5 * 12
        assert F.link_pa_executed(K, M, L, 4096) < F.gmp_flops_fig3(K, M, L) + 2 * 5 * 12
