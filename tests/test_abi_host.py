"""Host-side checks of the C ABI: the library loads, exports every function that
include/dpdmi.h declares, and rejects invalid arguments before any HIP call
(so these run without a GPU; no call here reaches a kernel launch)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2205_05158_amd as D
from paper_2205_05158_amd import _lib as L
import dpd_synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = C.c_void_p(0x100000)          # aligned, never dereferenced: validation fails first


def header_functions():
    txt = open(os.path.join(ROOT, "include", "dpdmi.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(\w+)\s*\(", txt, flags=re.M))
                  - {"if", "while", "for", "return", "sizeof"})


def test_library_exports_every_declared_function(dpdlib):
    names = header_functions()
    assert "dpd_forward" in names and "pa_gmp_forward" in names
    for n in names:
        assert hasattr(dpdlib, n), f"missing export {n}"
    assert set(names) == set(L.EXPORTS)
    assert D.dpd_version().endswith("gfx950")


def test_param_and_coeff_counts(dpdlib):
    for T, nl, H in [(4, 2, 20), (10, 3, 64), (16, 4, 128), (1, 1, 1)]:
        assert D.dpd_tdnn_param_count(D.tdnn_desc(T, nl, H)) == S.tdnn_param_count(T, nl, H)
    for K, M, Lg in [(5, 3, 2), (7, 5, 3), (9, 7, 4), (1, 0, 0)]:
        assert D.dpd_gmp_coeff_count(D.gmp_desc(K, M, Lg)) == S.gmp_coeff_count(K, M, Lg)
    assert D.dpd_gmp_coeff_count(D.gmp_desc(0, 1, 1)) == -1


def test_workspace_size_grows_with_problem(dpdlib):
    t = D.tdnn_desc(10, 3, 64)
    g = D.gmp_desc(7, 5, 3)
    a = D.dpd_workspace_size(t, g, D.make_batch([0, 1000]))
    b = D.dpd_workspace_size(t, g, D.make_batch([0, 100000]))
    assert 0 < a < b
    p = D.dpd_workspace_size(D.tdnn_desc(10, 3, 64, impl="plain"), g, D.make_batch([0, 1000]))
    assert p > 0


def _fwd(tdnn, batch, x=FAKE, w=FAKE, u=FAKE, ws=FAKE, nbytes=1 << 40):
    return L.lib().dpd_forward(C.byref(tdnn), C.byref(batch), x, w, u, ws, nbytes, None)


@pytest.mark.parametrize("desc,code", [
    (dict(taps=0), L.DPD_ERR_SHAPE), (dict(taps=33), L.DPD_ERR_SHAPE),
    (dict(hidden=0), L.DPD_ERR_SHAPE), (dict(n_hidden=9), L.DPD_ERR_SHAPE),
    (dict(residual=2), L.DPD_ERR_SHAPE), (dict(precision=7), L.DPD_ERR_SHAPE),
    (dict(impl=3), L.DPD_ERR_SHAPE),
    (dict(precision=L.DPD_BF16, impl=L.DPD_IMPL_PLAIN), L.DPD_ERR_UNSUPPORTED),
    (dict(hidden=129), L.DPD_ERR_UNSUPPORTED),     # wider than the tuned kernels
    (dict(n_hidden=5), L.DPD_ERR_UNSUPPORTED),     # deeper than the tuned kernels
])
def test_tdnn_descriptor_rejected(dpdlib, desc, code):
    base = dict(taps=10, n_hidden=3, hidden=64, residual=0, precision=0, impl=0)
    base.update(desc)
    t = L.TdnnDesc(**base)
    assert _fwd(t, D.make_batch([0, 100])) == code


@pytest.mark.parametrize("offsets,code", [
    ([1, 100], L.DPD_ERR_SHAPE),          # must start at 0
    ([0, 50, 50], L.DPD_ERR_SHAPE),       # empty stream
    ([0, 50, 20], L.DPD_ERR_SHAPE),       # decreasing
    ([0], L.DPD_ERR_SHAPE),               # no stream
])
def test_batch_rejected(dpdlib, offsets, code):
    assert _fwd(D.tdnn_desc(10, 3, 64), D.make_batch(offsets)) == code


def test_too_many_streams_rejected(dpdlib):
    off = np.arange(0, 130 * 10, 10)
    assert _fwd(D.tdnn_desc(10, 3, 64), D.make_batch(off)) == L.DPD_ERR_SHAPE


def test_null_and_alignment_and_workspace(dpdlib):
    t = D.tdnn_desc(10, 3, 64)
    b = D.make_batch([0, 100])
    assert _fwd(t, b, x=None) == L.DPD_ERR_NULL
    assert _fwd(t, b, u=None) == L.DPD_ERR_NULL
    assert _fwd(t, b, x=C.c_void_p(0x100004)) == L.DPD_ERR_ALIGN
    assert _fwd(t, b, nbytes=16) == L.DPD_ERR_WORKSPACE
    lib = L.lib()
    assert lib.dpd_forward(None, C.byref(b), FAKE, FAKE, FAKE, FAKE, 1 << 40, None) == L.DPD_ERR_NULL
    g = D.gmp_desc(7, 5, 3)
    assert lib.pa_gmp_forward(C.byref(g), C.byref(b), FAKE, FAKE, FAKE, None) == L.DPD_ERR_SHAPE  # u == y
    bad = D.gmp_desc(13, 1, 1)
    assert lib.pa_gmp_forward(C.byref(bad), C.byref(b), FAKE, FAKE, C.c_void_p(0x200000), None) == L.DPD_ERR_SHAPE
    # zero target gain is not a valid NMSE reference
    assert lib.cascade_nmse(C.byref(b), FAKE, FAKE, 0.0, 0.0, FAKE, FAKE, 1 << 40, None) == L.DPD_ERR_SHAPE
    # gradient without a loss output
    assert lib.dpd_cascade(C.byref(t), C.byref(g), C.byref(b), FAKE, FAKE, FAKE, 1.0, 0.0, None, None,
                           None, FAKE, None, FAKE, 1 << 40, None) == L.DPD_ERR_NULL
    # GMP orders beyond the tuned backward kernels' padded bound (rejected before any launch)
    g2 = D.gmp_desc(10, 2, 1)
    assert lib.dpd_backward(C.byref(t), C.byref(g2), C.byref(b), FAKE, FAKE, FAKE, 1.0, 0.0, FAKE, FAKE,
                            FAKE, 1 << 40, None) == L.DPD_ERR_UNSUPPORTED


def test_acpr_arguments_rejected(dpdlib):
    lib = L.lib()
    for n, nfft, hb in [(4096, 1000, 10), (100, 4096, 10), (8192, 4096, 700), (8192, 8192, 10)]:
        assert lib.cascade_acpr(FAKE, n, nfft, hb, FAKE, FAKE, FAKE, 1 << 40, None) == L.DPD_ERR_SHAPE
    assert lib.cascade_acpr(FAKE, 8192, 4096, 512, FAKE, FAKE, FAKE, 0, None) == L.DPD_ERR_WORKSPACE
    assert D.dpd_acpr_workspace_size(8192, 4096) > 0


def test_status_strings(dpdlib):
    for code in range(-7, 1):
        assert D.status_string(code).startswith("DPD_")
    assert "NONFINITE" in D.status_string(L.DPD_ERR_NONFINITE)


def test_nmse_status_host(dpdlib):
    """dpd_nmse_status reads host copies of the NMSE records (E, R, NMSE dB, count): a
    record with a non-finite count, E, R or an NMSE of NaN / +inf is DPD_ERR_NONFINITE;
    the exact match E = 0 (NMSE = -inf dB) is a finite result."""
    assert L.DPD_NMSE_FIELDS == 4
    good = np.array([[1.0, 2.0, -3.0103, 0.0], [0.0, 2.0, -np.inf, 0.0]], np.float32)
    assert D.dpd_nmse_status(good) == L.DPD_OK
    for bad_rec in ([1.0, 2.0, -3.0, 1.0], [np.nan, 2.0, np.nan, 0.0], [np.inf, 2.0, np.inf, 0.0],
                    [1.0, np.inf, -np.inf, 0.0], [1.0, 0.0, np.inf, 0.0], [0.0, 0.0, np.nan, 0.0]):
        recs = np.vstack([good, np.array(bad_rec, np.float32)])
        assert D.dpd_nmse_status(recs) == L.DPD_ERR_NONFINITE, bad_rec
    lib = L.lib()
    assert lib.dpd_nmse_status(None, 1) == L.DPD_ERR_NULL
    a = np.zeros(4, np.float32)
    assert lib.dpd_nmse_status(a.ctypes.data_as(C.POINTER(C.c_float)), 0) == L.DPD_ERR_SHAPE
    with pytest.raises(ValueError):
        D.dpd_nmse_status(np.zeros(6, np.float32))


def test_noalloc_nmse_arguments_rejected(dpdlib):
    """cascade_nmse_noalloc checks its arguments and the size of its static scratch
    before any HIP call."""
    lib = L.lib()
    f = lib.cascade_nmse_noalloc
    b = D.make_batch([0, 1000])
    assert f(C.byref(b), None, FAKE, 1.0, 0.0, FAKE, None) == L.DPD_ERR_NULL
    assert f(C.byref(b), FAKE, FAKE, 1.0, 0.0, None, None) == L.DPD_ERR_NULL
    assert f(C.byref(b), C.c_void_p(0x100004), FAKE, 1.0, 0.0, FAKE, None) == L.DPD_ERR_ALIGN
    assert f(C.byref(b), FAKE, FAKE, 0.0, 0.0, FAKE, None) == L.DPD_ERR_SHAPE
    assert f(C.byref(D.make_batch([0, 0])), FAKE, FAKE, 1.0, 0.0, FAKE, None) == L.DPD_ERR_SHAPE
    # tiles of 256 samples, one count per stream rounded up, plus one final-pass record per
    # 256 tiles of a stream
    cap = L.DPD_NOALLOC_NMSE_MAX_TILES * 256
    too_big = D.make_batch([0, cap + 1])
    assert f(C.byref(too_big), FAKE, FAKE, 1.0, 0.0, FAKE, None) == L.DPD_ERR_WORKSPACE
    m = L.DPD_NOALLOC_NMSE_MAX_TILES
    tiles = m - m // 257 + 1                      # tiles + ceil(tiles / 256) = m + 2
    assert tiles + -(-tiles // 256) > m
    over = D.make_batch([0, tiles * 256])
    assert f(C.byref(over), FAKE, FAKE, 1.0, 0.0, FAKE, None) == L.DPD_ERR_WORKSPACE


def test_symbol_mse_arguments_rejected(dpdlib):
    lib = L.lib()
    ws = L.dpd_symbol_mse_workspace_size(10000)
    assert ws >= 16 * 3
    assert L.dpd_symbol_mse_workspace_size(10000) < L.dpd_symbol_mse_workspace_size(10 ** 7)
    b = C.c_size_t(0)
    assert lib.dpd_symbol_mse_workspace_size(0, C.byref(b)) == L.DPD_ERR_SHAPE
    assert lib.dpd_symbol_mse_workspace_size(5, None) == L.DPD_ERR_NULL
    mse = lib.dpd_symbol_mse
    assert mse(0, FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 40, None) == L.DPD_ERR_SHAPE
    assert mse(10, None, FAKE, FAKE, None, FAKE, 1 << 40, None) == L.DPD_ERR_NULL
    assert mse(10, FAKE, FAKE, None, None, FAKE, 1 << 40, None) == L.DPD_ERR_NULL
    assert mse(10, FAKE, FAKE, FAKE, None, None, 1 << 40, None) == L.DPD_ERR_NULL
    assert mse(10, C.c_void_p(0x100004), FAKE, FAKE, None, FAKE, 1 << 40, None) == L.DPD_ERR_ALIGN
    assert mse(10, FAKE, FAKE, FAKE, None, C.c_void_p(0x100010), 1 << 40, None) == L.DPD_ERR_ALIGN
    assert mse(10, FAKE, C.c_void_p(0x200000), FAKE, FAKE, FAKE, 1 << 40, None) == L.DPD_ERR_SHAPE  # grad == z
    assert mse(10 ** 7, FAKE, FAKE, FAKE, None, FAKE, 256, None) == L.DPD_ERR_WORKSPACE


def test_tune_table_host(dpdlib):
    """Launch-shape table: defaults, install / read back / remove, range checks; the
    autotuner's argument checks (all host-side, before any HIP call)."""
    t = D.tdnn_desc(10, 3, 64)
    g = D.gmp_desc(7, 5, 3)
    b = D.make_batch([0, 1000, 5000], per_stream_params=True)
    b2 = D.make_batch([0, 1000, 5001], per_stream_params=True)
    d = D.dpd_tune_get(t, g, b)
    assert d["fwd_waves"] == 8 and d["bwd_wg_per_cu"] == 2 and d["gmp_tile"] == 256
    assert 1 <= d["fwd_wg_per_cu"] <= 2
    assert D.dpd_tune_get(D.tdnn_desc(16, 4, 128, precision="bf16"), D.gmp_desc(9, 7, 4), b)["fwd_waves"] == 12
    # generic shapes (the paper's FD-NN-sized core, odd sizes) have a tuned launch shape
    for shape in [(4, 1, 15), (3, 1, 7), (32, 4, 128), (17, 2, 100)]:
        for prec in ("fp32", "bf16"):
            assert D.dpd_tune_get(D.tdnn_desc(*shape, precision=prec), g, b)["fwd_waves"] in (8, 12)
    mine = dict(fwd_waves=12, fwd_wg_per_cu=3, bwd_wg_per_cu=1, gmp_tile=512)
    try:
        D.dpd_tune_set(t, g, b, mine)
        assert D.dpd_tune_get(t, g, b) == mine
        assert D.dpd_tune_get(t, g, b2) == d          # another batch signature
        assert D.dpd_tune_get(t, None, b) == d        # the forward-only key
    finally:
        D.dpd_tune_set(t, g, b, None)
    assert D.dpd_tune_get(t, g, b) == d
    lib = L.lib()
    for bad in [dict(mine, fwd_waves=10), dict(mine, fwd_wg_per_cu=0), dict(mine, fwd_wg_per_cu=5),
                dict(mine, bwd_wg_per_cu=3), dict(mine, gmp_tile=384)]:
        assert lib.dpd_tune_set(C.byref(t), C.byref(g), C.byref(b), C.byref(L.Tune(**bad))) == L.DPD_ERR_SHAPE
    plain = D.tdnn_desc(10, 3, 64, impl="plain")
    out = L.Tune()
    assert lib.dpd_tune_get(C.byref(plain), C.byref(g), C.byref(b), C.byref(out)) == L.DPD_ERR_UNSUPPORTED
    assert lib.dpd_tune_get(C.byref(t), C.byref(g), C.byref(b), None) == L.DPD_ERR_NULL

    def auto(tdnn=t, gmp=g, reps=2, out_=out, nbytes=1 << 40, x=FAKE):
        return lib.dpd_autotune(C.byref(tdnn), C.byref(gmp), C.byref(b), x, FAKE, FAKE, 1.0, 0.0, reps,
                                FAKE, nbytes, None, None if out_ is None else C.byref(out_))
    assert auto(reps=0) == L.DPD_ERR_SHAPE
    assert auto(out_=None) == L.DPD_ERR_NULL
    assert auto(x=None) == L.DPD_ERR_NULL
    assert auto(tdnn=plain) == L.DPD_ERR_UNSUPPORTED
    assert auto(gmp=D.gmp_desc(10, 2, 1)) == L.DPD_ERR_UNSUPPORTED
    assert auto(nbytes=16) == L.DPD_ERR_WORKSPACE


def test_adam_arguments_rejected(dpdlib):
    lib = L.lib()
    a, b, c, d = (C.c_void_p(0x100000 * k) for k in (1, 2, 3, 4))

    def adam(g=a, w=b, m=c, v=d, n=1000, step=1, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        return lib.dpd_adam_step(g, w, m, v, n, step, lr, b1, b2, eps, None)
    assert adam(g=None) == L.DPD_ERR_NULL and adam(v=None) == L.DPD_ERR_NULL
    assert adam(n=0) == L.DPD_ERR_SHAPE and adam(step=0) == L.DPD_ERR_SHAPE
    assert adam(b1=1.0) == L.DPD_ERR_SHAPE and adam(b2=-0.1) == L.DPD_ERR_SHAPE
    assert adam(eps=-1.0) == L.DPD_ERR_SHAPE and adam(lr=float("nan")) == L.DPD_ERR_SHAPE
    assert adam(w=C.c_void_p(0x100002)) == L.DPD_ERR_ALIGN
    assert adam(m=C.c_void_p(0x100000 + 400)) == L.DPD_ERR_SHAPE      # overlaps g
    assert adam(n=0x100000 // 4 + 1) == L.DPD_ERR_SHAPE                # now all overlap


def test_ls_fit_arguments_rejected(dpdlib):
    lib = L.lib()
    g = D.gmp_desc(7, 5, 3)
    b = D.make_batch([0, 5000])
    info = C.c_void_p(0x300000)

    def fit(gmp=g, y=FAKE, t=C.c_void_p(0x200000), ridge=0.0, coef=FAKE, inf=info, normal=None,
            nbytes=1 << 40, gr=1.0, gi=0.0):
        return lib.gmp_ls_fit(C.byref(gmp), C.byref(b), y, gr, gi, t, ridge, coef, inf, normal, FAKE,
                              nbytes, None)
    assert fit(y=None) == L.DPD_ERR_NULL and fit(inf=None) == L.DPD_ERR_NULL
    assert fit(ridge=-1.0) == L.DPD_ERR_SHAPE and fit(ridge=float("inf")) == L.DPD_ERR_SHAPE
    assert fit(gr=0.0) == L.DPD_ERR_SHAPE
    assert fit(normal=C.c_void_p(0x400008)) == L.DPD_ERR_ALIGN
    assert fit(nbytes=16) == L.DPD_ERR_WORKSPACE
    assert fit(gmp=D.gmp_desc(12, 15, 8)) == L.DPD_ERR_UNSUPPORTED      # J > 1024
    assert D.gmp_ls_workspace_size(g, b) > 0


def test_fdcnn_arguments_rejected(dpdlib):
    lib = L.lib()
    d = L.FdcnnDesc(384, 20, 2, 3)
    assert D.fdcnn_param_count(d) == 2 * 2 * 9 + 2 + 768 * 800 + 768
    for bad in [L.FdcnnDesc(401, 20, 2, 3), L.FdcnnDesc(384, 40, 2, 3), L.FdcnnDesc(384, 20, 2, 4),
                L.FdcnnDesc(384, 20, 5, 3), L.FdcnnDesc(0, 20, 2, 3)]:
        assert D.fdcnn_param_count(bad) == -1
        assert lib.fdcnn_forward(C.byref(bad), 4, FAKE, FAKE, C.c_void_p(0x200000), FAKE, 1 << 40,
                                 None) == L.DPD_ERR_UNSUPPORTED
    assert lib.fdcnn_forward(C.byref(d), 0, FAKE, FAKE, C.c_void_p(0x200000), FAKE, 1 << 40, None) == L.DPD_ERR_SHAPE
    assert lib.fdcnn_forward(C.byref(d), 4, FAKE, FAKE, FAKE, FAKE, 1 << 40, None) == L.DPD_ERR_SHAPE   # s == out
    assert lib.fdcnn_forward(C.byref(d), 4, None, FAKE, FAKE, FAKE, 1 << 40, None) == L.DPD_ERR_NULL
    assert lib.fdcnn_backward(C.byref(d), 4, FAKE, FAKE, FAKE, FAKE, FAKE, 16, None) == L.DPD_ERR_WORKSPACE
    assert lib.fdcnn_backward(C.byref(d), 4, FAKE, FAKE, C.c_void_p(0x100004), FAKE, FAKE, 1 << 40,
                              None) == L.DPD_ERR_ALIGN
    assert D.fdcnn_workspace_size(d, 100) > D.fdcnn_workspace_size(d, 10)


def test_downlink_arguments_rejected(dpdlib):
    lib = L.lib()
    OUT = C.c_void_p(0x200000)
    # FFT: sizes are powers of two in [2, 4096]
    for n in (0, 1, 3, 96, 8192):
        assert lib.ofdm_fft(n, 4, 0, FAKE, OUT, None) == L.DPD_ERR_SHAPE
    assert lib.ofdm_fft(64, 0, 0, FAKE, OUT, None) == L.DPD_ERR_SHAPE
    assert lib.ofdm_fft(64, 4, 2, FAKE, OUT, None) == L.DPD_ERR_SHAPE
    assert lib.ofdm_fft(64, 4, 0, None, OUT, None) == L.DPD_ERR_NULL
    assert lib.ofdm_fft(64, 4, 0, C.c_void_p(0x100004), OUT, None) == L.DPD_ERR_ALIGN
    # FD-NN: the paper's network (U = 8, L4 = 3, D = 15, one hidden layer)
    d = L.fdnn_desc(4096, 8, 3, 15, 1)
    assert D.FdNn.__name__ and L.fdnn_param_count(d) == 15 * 64 + 15 + 16 * 15 + 16
    assert L.fdnn_param_count(L.fdnn_desc(64, 2, 1, 4, 2)) == 4 * 8 + 4 + 4 * 4 + 4 + 4 * 4 + 4
    for bad in [L.fdnn_desc(4096, 9, 3, 15, 1), L.fdnn_desc(4096, 8, 4, 15, 1), L.fdnn_desc(4096, 8, 3, 33, 1),
                L.fdnn_desc(4096, 8, 3, 15, 3), L.fdnn_desc(4000, 8, 3, 15, 1), L.fdnn_desc(4096, 0, 3, 15, 1)]:
        assert L.fdnn_param_count(bad) == -1
        assert lib.fdnn_forward(C.byref(bad), 2, FAKE, FAKE, OUT, FAKE, 1 << 40, None) == L.DPD_ERR_UNSUPPORTED
    assert lib.fdnn_forward(C.byref(d), 0, FAKE, FAKE, OUT, FAKE, 1 << 40, None) == L.DPD_ERR_SHAPE
    assert lib.fdnn_forward(C.byref(d), 2, None, FAKE, OUT, FAKE, 1 << 40, None) == L.DPD_ERR_NULL
    assert lib.fdnn_forward(C.byref(d), 2, FAKE, FAKE, OUT, FAKE, 16, None) == L.DPD_ERR_WORKSPACE
    assert lib.fdnn_backward(C.byref(d), 2, FAKE, FAKE, FAKE, C.c_void_p(0x100002), FAKE, 1 << 40,
                             None) == L.DPD_ERR_ALIGN
    assert L.fdnn_workspace_size(d, 20) > L.fdnn_workspace_size(d, 2)
    # link: U <= 8, B <= 256, T <= 64, square QAM, GMP orders in range
    pa = L.GmpDesc(7, 3, 1)
    ok = L.link_desc(4096, 384, 8, 32, 10, 256, pa)
    assert L.zf_workspace_size(ok, 3) >= 3 * 4096 * 8
    cases = [(L.link_desc(4096, 384, 9, 32, 10, 256, pa), L.DPD_ERR_UNSUPPORTED),
             (L.link_desc(4096, 384, 8, 257, 10, 256, pa), L.DPD_ERR_UNSUPPORTED),
             (L.link_desc(4096, 384, 8, 32, 65, 256, pa), L.DPD_ERR_UNSUPPORTED),
             (L.link_desc(4096, 384, 8, 32, 10, 200, pa), L.DPD_ERR_SHAPE),
             (L.link_desc(4096, 385, 8, 32, 10, 256, pa), L.DPD_ERR_SHAPE),
             (L.link_desc(4096, 4096, 8, 32, 10, 256, pa), L.DPD_ERR_SHAPE),
             (L.link_desc(3000, 384, 8, 32, 10, 256, pa), L.DPD_ERR_SHAPE),
             (L.link_desc(4096, 384, 8, 32, 10, 256, L.GmpDesc(13, 3, 1)), L.DPD_ERR_SHAPE),
             (L.link_desc(16, 8, 2, 4, 2, 16, L.GmpDesc(3, 15, 1)), L.DPD_ERR_SHAPE),      # M + L >= N
             (L.link_desc(4096, 384, 8, 32, 10, 256, pa, L.GmpDesc(3, 16, 0)), L.DPD_ERR_SHAPE)]
    for desc, code in cases:
        assert lib.zf_precoder(C.byref(desc), 1, FAKE, C.c_float(1.0), 0, OUT, FAKE, FAKE, 1 << 40, None) == code
        assert lib.ofdm_link(C.byref(desc), 2, 1, FAKE, FAKE, FAKE, C.c_float(1.0), C.c_float(0.0), FAKE, FAKE,
                             None, FAKE, None, FAKE, FAKE, 1 << 40, None) == code
    assert lib.zf_precoder(C.byref(ok), 1, FAKE, C.c_float(0.0), 0, OUT, FAKE, FAKE, 1 << 40, None) == L.DPD_ERR_SHAPE
    assert lib.zf_precoder(C.byref(ok), 2, FAKE, C.c_float(1.0), 0, OUT, FAKE, FAKE, 16, None) == L.DPD_ERR_WORKSPACE
    assert lib.zf_precoder(C.byref(ok), 1, FAKE, C.c_float(1.0), 2, OUT, FAKE, FAKE, 1 << 40, None) == L.DPD_ERR_SHAPE
    assert lib.ofdm_precode(C.byref(ok), 4, 0, FAKE, FAKE, FAKE, 0, OUT, None) == L.DPD_ERR_SHAPE
    assert lib.ofdm_precode(C.byref(ok), 4, 1, FAKE, FAKE, FAKE, 2, OUT, None) == L.DPD_ERR_SHAPE
    # a DPD in the descriptor needs its coefficients; a zero gain cannot be equalised
    withdpd = L.link_desc(4096, 384, 8, 32, 10, 256, pa, L.GmpDesc(5, 2, 1))
    assert lib.ofdm_link(C.byref(withdpd), 2, 1, FAKE, None, FAKE, C.c_float(1.0), C.c_float(0.0), FAKE, FAKE,
                         None, FAKE, None, FAKE, FAKE, 1 << 40, None) == L.DPD_ERR_NULL
    assert lib.ofdm_link(C.byref(ok), 2, 1, FAKE, None, FAKE, C.c_float(0.0), C.c_float(0.0), FAKE, FAKE,
                         None, FAKE, None, FAKE, FAKE, 1 << 40, None) == L.DPD_ERR_SHAPE
    assert lib.ofdm_link(C.byref(ok), 2, 1, FAKE, None, FAKE, C.c_float(1.0), C.c_float(0.0), FAKE, FAKE,
                         None, FAKE, None, FAKE, FAKE, 64, None) == L.DPD_ERR_WORKSPACE
    assert L.link_workspace_size(ok, 20, 10) > L.link_workspace_size(ok, 2, 1)
    # reverse mode: no DPD in the descriptor, x and g_x distinct
    assert lib.ofdm_link_backward(C.byref(withdpd), 2, 1, FAKE, FAKE, C.c_float(1.0), C.c_float(0.0), FAKE, FAKE,
                                  FAKE, OUT, FAKE, 1 << 40, None) == L.DPD_ERR_UNSUPPORTED
    assert lib.ofdm_link_backward(C.byref(ok), 2, 1, FAKE, FAKE, C.c_float(1.0), C.c_float(0.0), FAKE, FAKE,
                                  FAKE, FAKE, FAKE, 1 << 40, None) == L.DPD_ERR_SHAPE
    assert lib.ofdm_link_backward(C.byref(ok), 2, 1, FAKE, FAKE, C.c_float(1.0), C.c_float(0.0), FAKE, FAKE,
                                  None, OUT, FAKE, 1 << 40, None) == L.DPD_ERR_NULL
    assert lib.ofdm_precode_backward(C.byref(ok), 2, 1, FAKE, FAKE, FAKE, 3, OUT, None) == L.DPD_ERR_SHAPE


def test_clip_pa_arguments_rejected(dpdlib):
    lib = L.lib()
    Y = C.c_void_p(0x300000)
    for n, a in [(0, 1.0), (-5, 1.0), (10, 0.0), (10, -1.0), (10, float("nan")), (10, float("inf"))]:
        assert lib.pa_clip_forward(n, FAKE, a, Y, None) == L.DPD_ERR_SHAPE
    assert lib.pa_clip_forward(10, None, 1.0, Y, None) == L.DPD_ERR_NULL
    assert lib.pa_clip_forward(10, C.c_void_p(0x100004), 1.0, Y, None) == L.DPD_ERR_ALIGN
    t = D.tdnn_desc(10, 3, 64)
    b = D.make_batch([0, 100])

    def casc(a=1.0, dw=None, loss=None, nbytes=1 << 40, tdnn=t, x=FAKE):
        return lib.dpd_cascade_clip(C.byref(tdnn), C.byref(b), x, FAKE, a, 1.0, 0.0, None, None, None, dw,
                                    loss, FAKE, nbytes, None)
    assert casc(a=0.0) == L.DPD_ERR_SHAPE
    assert casc(a=float("nan")) == L.DPD_ERR_SHAPE
    assert casc(x=None) == L.DPD_ERR_NULL
    assert casc(dw=FAKE) == L.DPD_ERR_NULL                 # gradient without a loss output
    assert casc(nbytes=16) == L.DPD_ERR_WORKSPACE
    assert casc(tdnn=D.tdnn_desc(10, 3, 200)) == L.DPD_ERR_UNSUPPORTED
    # the clip cascade needs no GMP table: its workspace is the forward-only one
    assert D.dpd_workspace_size(t, None, b) < D.dpd_workspace_size(t, D.gmp_desc(7, 5, 3), b)
