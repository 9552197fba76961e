"""Checks of the seeded input generators (shapes, statistics, reproducibility)."""
import numpy as np

import dpd_synth as D


def test_qam_unit_energy_and_grid():
    pts = D.qam_constellation(64)
    assert pts.size == 64
    np.testing.assert_allclose(np.mean(np.abs(pts) ** 2), 1.0, rtol=1e-14)
    np.testing.assert_allclose(np.sort(np.unique(np.round(pts.real * np.sqrt(42), 9))),
                               [-7, -5, -3, -1, 1, 3, 5, 7])


def test_ofdm_unit_rms_and_occupied_band():
    x = D.ofdm_signal(2048, 1200, 8, 64, np.random.default_rng(0))
    assert x.size == 16384
    np.testing.assert_allclose(np.sqrt(np.mean(np.abs(x) ** 2)), 1.0, rtol=1e-12)
    X = np.fft.fft(x[:2048])
    p = np.abs(X) ** 2
    active = np.r_[1:601, 2048 - 600:2048]
    assert p[0] < 1e-20 * p.max()                       # DC null
    assert p[601:2048 - 600].max() < 1e-20 * p.max()    # guard band empty
    assert p[active].min() > 0


def test_papr_clip_reaches_target():
    wl = D.WORKLOADS["bf16_16m"]
    x = D.ofdm_signal(4096, 1024, 64, 64, np.random.default_rng(0))
    assert D.papr_db(x) > 10.5
    y = D.papr_clip(x, 10.0)
    assert abs(D.papr_db(y) - 10.0) <= 0.1
    np.testing.assert_allclose(np.mean(np.abs(y) ** 2), 1.0, rtol=1e-12)
    assert wl.papr_target_db == 10.0


def test_stream_lengths_log_uniform_range_and_seed():
    a = D.stream_lengths(64)
    b = D.stream_lengths(64)
    np.testing.assert_array_equal(a, b)
    assert a.min() >= 2 ** 14 and a.max() <= 2 ** 20
    assert 100_000 < a.mean() < 400_000


def test_parameter_counts():
    assert D.tdnn_param_count(4, 2, 20) == 882
    assert D.tdnn_param_count(10, 3, 64) == 11714
    assert D.tdnn_param_count(16, 4, 128) == 60162
    assert D.gmp_coeff_count(5, 3, 2) == 84
    assert D.gmp_coeff_count(7, 5, 3) == 258
    assert D.gmp_coeff_count(9, 7, 4) == 584


def test_gmp_coefficient_statistics_and_linear_term():
    c = D.gmp_coefficients(7, 5, 3, seed=2)
    z = c[:, 0] + 1j * c[:, 1]
    assert z[0] == 1.0
    assert c.dtype == np.float32 and c.shape == (258, 2)
    np.testing.assert_array_equal(c, D.gmp_coefficients(7, 5, 3, seed=2))


def test_xavier_bounds_and_zero_bias():
    w = D.xavier_tdnn(10, 3, 64, seed=1)
    W1 = w[:64 * 50]
    lim = np.sqrt(6 / (50 + 64))
    assert np.abs(W1).max() <= lim and np.abs(W1).max() > 0.9 * lim
    np.testing.assert_array_equal(w[64 * 50:64 * 51], 0)


def test_workload_shapes():
    inp = D.make_workload("parity_16k")
    assert inp.x.shape == (16384, 2) and inp.x.dtype == np.float32
    assert list(inp.offsets) == [0, 16384]
    inp = D.make_workload("train_1m_8f", max_len=1000)
    assert list(inp.offsets) == [i * 1000 for i in range(9)]
    inp = D.make_workload("batched_64s", n_streams=3, max_len=5000)
    assert inp.w.shape == (3, 11714) and inp.coef.shape == (3, 258, 2)
    assert inp.offsets[-1] == inp.x.shape[0]


def test_workload_stream_selection_without_truncation():
    inp = D.make_workload("train_1m_8f", n_streams=1)
    assert list(inp.offsets) == [0, 131072]
    full = D.make_workload("train_1m_8f")
    np.testing.assert_array_equal(full.x[:131072], inp.x)
