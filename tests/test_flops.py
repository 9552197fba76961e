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
