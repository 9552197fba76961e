"""ctypes binding of libdpdmi.so (include/dpdmi.h).

Argument marshalling only: every entry point here has the name of the C function
it calls, takes torch device tensors where the C function takes device pointers,
and raises RuntimeError with the library's status string when the call fails.
The library itself must be built (python -m paper_2205_05158_amd.build); there is
no fallback of any kind when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpdmi.so")

DPD_OK = 0
DPD_ERR_NULL, DPD_ERR_SHAPE, DPD_ERR_UNSUPPORTED, DPD_ERR_WORKSPACE, DPD_ERR_LAUNCH, DPD_ERR_ALIGN, \
    DPD_ERR_NONFINITE = -1, -2, -3, -4, -5, -6, -7
DPD_NMSE_FIELDS = 4    # (E, R, NMSE dB, non-finite count) per NMSE record
DPD_FP32, DPD_BF16 = 0, 1
DPD_IMPL_TUNED, DPD_IMPL_PLAIN = 0, 1
DPD_MAX_STREAMS = 128


class TdnnDesc(C.Structure):
    _fields_ = [("taps", C.c_int32), ("n_hidden", C.c_int32), ("hidden", C.c_int32),
                ("residual", C.c_int32), ("precision", C.c_int32), ("impl", C.c_int32)]


class GmpDesc(C.Structure):
    _fields_ = [("K", C.c_int32), ("M", C.c_int32), ("L", C.c_int32)]


class Batch(C.Structure):
    _fields_ = [("n_streams", C.c_int32), ("per_stream_params", C.c_int32),
                ("offsets_host", C.POINTER(C.c_int64))]


class FdcnnDesc(C.Structure):
    _fields_ = [("n_d", C.c_int32), ("side", C.c_int32), ("n_conv", C.c_int32), ("kc", C.c_int32)]


class FdnnDesc(C.Structure):
    _fields_ = [("n_fft", C.c_int32), ("users", C.c_int32), ("memory", C.c_int32), ("hidden", C.c_int32),
                ("n_hidden", C.c_int32)]


class LinkDesc(C.Structure):
    _fields_ = [("n_fft", C.c_int32), ("n_data", C.c_int32), ("users", C.c_int32), ("antennas", C.c_int32),
                ("taps", C.c_int32), ("qam", C.c_int32), ("pa", GmpDesc), ("dpd", GmpDesc)]


class Tune(C.Structure):
    _fields_ = [("fwd_waves", C.c_int32), ("fwd_wg_per_cu", C.c_int32),
                ("bwd_wg_per_cu", C.c_int32), ("gmp_tile", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None
_lock = threading.Lock()

_P = C.c_void_p
_SIGS = {
    "dpd_tdnn_param_count": (C.c_int64, [C.POINTER(TdnnDesc)]),
    "dpd_gmp_coeff_count": (C.c_int64, [C.POINTER(GmpDesc)]),
    "dpd_workspace_size": (C.c_int, [C.POINTER(TdnnDesc), C.POINTER(GmpDesc), C.POINTER(Batch),
                                     C.POINTER(C.c_size_t)]),
    "dpd_forward": (C.c_int, [C.POINTER(TdnnDesc), C.POINTER(Batch), _P, _P, _P, _P, C.c_size_t, _P]),
    "pa_gmp_forward": (C.c_int, [C.POINTER(GmpDesc), C.POINTER(Batch), _P, _P, _P, _P]),
    "cascade_nmse": (C.c_int, [C.POINTER(Batch), _P, _P, C.c_float, C.c_float, _P, _P, C.c_size_t, _P]),
    "dpd_backward": (C.c_int, [C.POINTER(TdnnDesc), C.POINTER(GmpDesc), C.POINTER(Batch), _P, _P, _P,
                               C.c_float, C.c_float, _P, _P, _P, C.c_size_t, _P]),
    "dpd_cascade": (C.c_int, [C.POINTER(TdnnDesc), C.POINTER(GmpDesc), C.POINTER(Batch), _P, _P, _P,
                              C.c_float, C.c_float, _P, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "pa_clip_forward": (C.c_int, [C.c_int64, _P, C.c_float, _P, _P]),
    "dpd_cascade_clip": (C.c_int, [C.POINTER(TdnnDesc), C.POINTER(Batch), _P, _P, C.c_float, C.c_float,
                                   C.c_float, _P, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "dpd_tune_get": (C.c_int, [C.POINTER(TdnnDesc), C.POINTER(GmpDesc), C.POINTER(Batch), C.POINTER(Tune)]),
    "dpd_tune_set": (C.c_int, [C.POINTER(TdnnDesc), C.POINTER(GmpDesc), C.POINTER(Batch), C.POINTER(Tune)]),
    "dpd_autotune": (C.c_int, [C.POINTER(TdnnDesc), C.POINTER(GmpDesc), C.POINTER(Batch), _P, _P, _P,
                               C.c_float, C.c_float, C.c_int32, _P, C.c_size_t, _P, C.POINTER(Tune)]),
    "dpd_nmse_status": (C.c_int, [C.POINTER(C.c_float), C.c_int64]),
    "cascade_nmse_noalloc": (C.c_int, [C.POINTER(Batch), _P, _P, C.c_float, C.c_float, _P, _P]),
    "dpd_symbol_mse_workspace_size": (C.c_int, [C.c_int64, C.POINTER(C.c_size_t)]),
    "dpd_symbol_mse": (C.c_int, [C.c_int64, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "dpd_adam_step": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.c_int32, C.c_double, C.c_double,
                                C.c_double, C.c_double, _P]),
    "gmp_ls_workspace_size": (C.c_int, [C.POINTER(GmpDesc), C.POINTER(Batch), C.POINTER(C.c_size_t)]),
    "gmp_ls_fit": (C.c_int, [C.POINTER(GmpDesc), C.POINTER(Batch), _P, C.c_float, C.c_float, _P, C.c_double,
                             _P, _P, _P, _P, C.c_size_t, _P]),
    "fdcnn_param_count": (C.c_int64, [C.POINTER(FdcnnDesc)]),
    "fdcnn_workspace_size": (C.c_int, [C.POINTER(FdcnnDesc), C.c_int64, C.POINTER(C.c_size_t)]),
    "fdcnn_forward": (C.c_int, [C.POINTER(FdcnnDesc), C.c_int64, _P, _P, _P, _P, C.c_size_t, _P]),
    "fdcnn_backward": (C.c_int, [C.POINTER(FdcnnDesc), C.c_int64, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "ofdm_fft": (C.c_int, [C.c_int32, C.c_int64, C.c_int32, _P, _P, _P]),
    "fdnn_param_count": (C.c_int64, [C.POINTER(FdnnDesc)]),
    "fdnn_workspace_size": (C.c_int, [C.POINTER(FdnnDesc), C.c_int64, C.POINTER(C.c_size_t)]),
    "fdnn_forward": (C.c_int, [C.POINTER(FdnnDesc), C.c_int64, _P, _P, _P, _P, C.c_size_t, _P]),
    "fdnn_backward": (C.c_int, [C.POINTER(FdnnDesc), C.c_int64, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "zf_workspace_size": (C.c_int, [C.POINTER(LinkDesc), C.c_int32, C.POINTER(C.c_size_t)]),
    "zf_precoder": (C.c_int, [C.POINTER(LinkDesc), C.c_int32, _P, C.c_float, C.c_int32, _P, _P, _P, C.c_size_t,
                              _P]),
    "ofdm_precode": (C.c_int, [C.POINTER(LinkDesc), C.c_int32, C.c_int32, _P, _P, _P, C.c_int32, _P, _P]),
    "link_workspace_size": (C.c_int, [C.POINTER(LinkDesc), C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "ofdm_link": (C.c_int, [C.POINTER(LinkDesc), C.c_int32, C.c_int32, _P, _P, _P, C.c_float, C.c_float, _P, _P,
                            _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "ofdm_link_backward": (C.c_int, [C.POINTER(LinkDesc), C.c_int32, C.c_int32, _P, _P, C.c_float, C.c_float, _P,
                                     _P, _P, _P, _P, C.c_size_t, _P]),
    "ofdm_precode_backward": (C.c_int, [C.POINTER(LinkDesc), C.c_int32, C.c_int32, _P, _P, _P, C.c_int32, _P,
                                        _P]),
    "cascade_acpr": (C.c_int, [_P, C.c_int64, C.c_int32, C.c_int32, _P, _P, _P, C.c_size_t, _P]),
    "dpd_acpr_workspace_size": (C.c_size_t, [C.c_int64, C.c_int32]),
    "dpd_profile_enable": (C.c_int, [C.c_int32]),
    "dpd_profile_report": (C.c_int32, [C.c_char_p, C.c_size_t]),
    "dpd_status_string": (C.c_char_p, [C.c_int]),
    "dpd_version": (C.c_char_p, []),
}
EXPORTS = tuple(_SIGS)


def lib():
    """Load libdpdmi.so once; raise if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -m paper_2205_05158_amd.build`")
            h = C.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                fn = getattr(h, name)
                fn.restype = res
                fn.argtypes = args
            _lib = h
        return _lib


def status_string(code: int) -> str:
    return lib().dpd_status_string(code).decode()


def _check(code: int, what: str):
    if code != DPD_OK:
        raise RuntimeError(f"{what}: {status_string(code)}")


# ------------------------------------------------------------------ marshalling
def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)


def make_batch(offsets, per_stream_params: bool = False):
    """Batch descriptor; the returned object keeps the host offsets alive."""
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    b = Batch(int(off.size - 1), int(bool(per_stream_params)),
              off.ctypes.data_as(C.POINTER(C.c_int64)))
    b._keep = off
    return b


def tdnn_desc(taps, n_hidden, hidden, residual=False, precision="fp32", impl="tuned"):
    prec = {"fp32": DPD_FP32, "bf16": DPD_BF16}[precision] if isinstance(precision, str) else precision
    im = {"tuned": DPD_IMPL_TUNED, "plain": DPD_IMPL_PLAIN}[impl] if isinstance(impl, str) else impl
    return TdnnDesc(taps, n_hidden, hidden, int(bool(residual)), prec, im)


def gmp_desc(K, M, L):
    return GmpDesc(K, M, L)


# ------------------------------------------------------------------ entry points
def dpd_tdnn_param_count(tdnn: TdnnDesc) -> int:
    return lib().dpd_tdnn_param_count(C.byref(tdnn))


def dpd_gmp_coeff_count(gmp: GmpDesc) -> int:
    return lib().dpd_gmp_coeff_count(C.byref(gmp))


def dpd_workspace_size(tdnn, gmp, batch) -> int:
    n = C.c_size_t(0)
    _check(lib().dpd_workspace_size(C.byref(tdnn) if tdnn is not None else None,
                                    C.byref(gmp) if gmp is not None else None,
                                    C.byref(batch), C.byref(n)), "dpd_workspace_size")
    return n.value


def dpd_forward(tdnn, batch, x, w, u, workspace, stream=None):
    _check(lib().dpd_forward(C.byref(tdnn), C.byref(batch), _ptr(x), _ptr(w), _ptr(u),
                             _ptr(workspace), workspace.numel() * workspace.element_size(),
                             _stream(stream)), "dpd_forward")


def pa_gmp_forward(gmp, batch, u, coef, y, stream=None):
    _check(lib().pa_gmp_forward(C.byref(gmp), C.byref(batch), _ptr(u), _ptr(coef), _ptr(y),
                                _stream(stream)), "pa_gmp_forward")


def cascade_nmse(batch, y, x, g, out, workspace, stream=None):
    g = complex(g)
    _check(lib().cascade_nmse(C.byref(batch), _ptr(y), _ptr(x), g.real, g.imag, _ptr(out),
                              _ptr(workspace), workspace.numel() * workspace.element_size(),
                              _stream(stream)), "cascade_nmse")


def dpd_nmse_status(records) -> int:
    """Status of NMSE records (host array-like [n][DPD_NMSE_FIELDS] or flat): DPD_OK or
    DPD_ERR_NONFINITE.  Runs on the host; copy device records first."""
    a = np.ascontiguousarray(np.asarray(records, dtype=np.float32).reshape(-1))
    if a.size == 0 or a.size % DPD_NMSE_FIELDS:
        raise ValueError("records must hold whole DPD_NMSE_FIELDS-float records")
    code = lib().dpd_nmse_status(a.ctypes.data_as(C.POINTER(C.c_float)), a.size // DPD_NMSE_FIELDS)
    if code not in (DPD_OK, DPD_ERR_NONFINITE):
        _check(code, "dpd_nmse_status")
    return code


def dpd_symbol_mse_workspace_size(n) -> int:
    b = C.c_size_t(0)
    _check(lib().dpd_symbol_mse_workspace_size(int(n), C.byref(b)), "dpd_symbol_mse_workspace_size")
    return b.value


def dpd_symbol_mse(n, z, t, out, grad, workspace, stream=None):
    _check(lib().dpd_symbol_mse(int(n), _ptr(z), _ptr(t), _ptr(out), _ptr(grad), _ptr(workspace),
                                workspace.numel() * workspace.element_size(), _stream(stream)),
           "dpd_symbol_mse")


DPD_NOALLOC_NMSE_MAX_TILES = 1 << 18


def cascade_nmse_noalloc(batch, y, x, g, out, stream=None):
    g = complex(g)
    _check(lib().cascade_nmse_noalloc(C.byref(batch), _ptr(y), _ptr(x), g.real, g.imag, _ptr(out),
                                      _stream(stream)), "cascade_nmse_noalloc")


def dpd_backward(tdnn, gmp, batch, x, w, coef, g, dw, loss, workspace, stream=None):
    g = complex(g)
    _check(lib().dpd_backward(C.byref(tdnn), C.byref(gmp), C.byref(batch), _ptr(x), _ptr(w),
                              _ptr(coef), g.real, g.imag, _ptr(dw), _ptr(loss), _ptr(workspace),
                              workspace.numel() * workspace.element_size(), _stream(stream)),
           "dpd_backward")


def dpd_cascade(tdnn, gmp, batch, x, w, coef, g, u, y, nmse, dw, loss, workspace, stream=None):
    g = complex(g)
    _check(lib().dpd_cascade(C.byref(tdnn), C.byref(gmp), C.byref(batch), _ptr(x), _ptr(w),
                             _ptr(coef), g.real, g.imag, _ptr(u), _ptr(y), _ptr(nmse), _ptr(dw),
                             _ptr(loss), _ptr(workspace),
                             workspace.numel() * workspace.element_size(), _stream(stream)),
           "dpd_cascade")


def pa_clip_forward(n, u, a_clip, y, stream=None):
    _check(lib().pa_clip_forward(int(n), _ptr(u), float(a_clip), _ptr(y), _stream(stream)), "pa_clip_forward")


def dpd_cascade_clip(tdnn, batch, x, w, a_clip, g, u, y, nmse, dw, loss, workspace, stream=None):
    g = complex(g)
    _check(lib().dpd_cascade_clip(C.byref(tdnn), C.byref(batch), _ptr(x), _ptr(w), float(a_clip), g.real,
                                  g.imag, _ptr(u), _ptr(y), _ptr(nmse), _ptr(dw), _ptr(loss), _ptr(workspace),
                                  workspace.numel() * workspace.element_size(), _stream(stream)),
           "dpd_cascade_clip")


def _gref(gmp):
    return None if gmp is None else C.byref(gmp)


def dpd_tune_get(tdnn, gmp, batch) -> dict:
    t = Tune()
    _check(lib().dpd_tune_get(C.byref(tdnn), _gref(gmp), C.byref(batch), C.byref(t)), "dpd_tune_get")
    return t.as_dict()


def dpd_tune_set(tdnn, gmp, batch, tune) -> None:
    """tune: dict with the four dpd_tune fields, or None to remove the entry."""
    t = None if tune is None else C.byref(Tune(**{k: int(v) for k, v in tune.items()}))
    _check(lib().dpd_tune_set(C.byref(tdnn), _gref(gmp), C.byref(batch), t), "dpd_tune_set")


def dpd_autotune(tdnn, gmp, batch, x, w, coef, g, reps, workspace, stream=None) -> dict:
    g = complex(g)
    t = Tune()
    _check(lib().dpd_autotune(C.byref(tdnn), C.byref(gmp), C.byref(batch), _ptr(x), _ptr(w), _ptr(coef),
                              g.real, g.imag, int(reps), _ptr(workspace),
                              workspace.numel() * workspace.element_size(), _stream(stream), C.byref(t)),
           "dpd_autotune")
    return t.as_dict()


def dpd_adam_step(grad, w, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    n = w.numel()
    for t in (grad, m, v):
        if t.numel() != n:
            raise ValueError("grad, w, m and v must have the same number of elements")
    _check(lib().dpd_adam_step(_ptr(grad), _ptr(w), _ptr(m), _ptr(v), n, int(step), lr, beta1, beta2,
                               eps, _stream(stream)), "dpd_adam_step")


def gmp_ls_workspace_size(gmp, batch) -> int:
    n = C.c_size_t(0)
    _check(lib().gmp_ls_workspace_size(C.byref(gmp), C.byref(batch), C.byref(n)), "gmp_ls_workspace_size")
    return n.value


def gmp_ls_fit(gmp, batch, y, g, t, ridge, coef, info, normal, workspace, stream=None):
    g = complex(g)
    _check(lib().gmp_ls_fit(C.byref(gmp), C.byref(batch), _ptr(y), g.real, g.imag, _ptr(t), float(ridge),
                            _ptr(coef), _ptr(info), _ptr(normal), _ptr(workspace),
                            workspace.numel() * workspace.element_size(), _stream(stream)), "gmp_ls_fit")


def fdcnn_param_count(desc) -> int:
    return lib().fdcnn_param_count(C.byref(desc))


def fdcnn_workspace_size(desc, n_items) -> int:
    n = C.c_size_t(0)
    _check(lib().fdcnn_workspace_size(C.byref(desc), int(n_items), C.byref(n)), "fdcnn_workspace_size")
    return n.value


def fdcnn_forward(desc, n_items, s, w, out, workspace, stream=None):
    _check(lib().fdcnn_forward(C.byref(desc), int(n_items), _ptr(s), _ptr(w), _ptr(out), _ptr(workspace),
                               workspace.numel() * workspace.element_size(), _stream(stream)), "fdcnn_forward")


def fdcnn_backward(desc, n_items, s, w, g_out, dw, workspace, stream=None):
    _check(lib().fdcnn_backward(C.byref(desc), int(n_items), _ptr(s), _ptr(w), _ptr(g_out), _ptr(dw),
                                _ptr(workspace), workspace.numel() * workspace.element_size(),
                                _stream(stream)), "fdcnn_backward")


def _nbytes(t) -> int:
    return t.numel() * t.element_size()


def ofdm_fft(n_fft, rows, inverse, x, out, stream=None):
    _check(lib().ofdm_fft(int(n_fft), int(rows), int(bool(inverse)), _ptr(x), _ptr(out), _stream(stream)),
           "ofdm_fft")


def fdnn_desc(n_fft, users, memory, hidden, n_hidden) -> FdnnDesc:
    return FdnnDesc(int(n_fft), int(users), int(memory), int(hidden), int(n_hidden))


def fdnn_param_count(desc) -> int:
    return lib().fdnn_param_count(C.byref(desc))


def fdnn_workspace_size(desc, n_sym) -> int:
    n = C.c_size_t(0)
    _check(lib().fdnn_workspace_size(C.byref(desc), int(n_sym), C.byref(n)), "fdnn_workspace_size")
    return n.value


def fdnn_forward(desc, n_sym, s, w, out, workspace, stream=None):
    _check(lib().fdnn_forward(C.byref(desc), int(n_sym), _ptr(s), _ptr(w), _ptr(out), _ptr(workspace),
                              _nbytes(workspace), _stream(stream)), "fdnn_forward")


def fdnn_backward(desc, n_sym, s, w, g_out, dw, workspace, stream=None):
    _check(lib().fdnn_backward(C.byref(desc), int(n_sym), _ptr(s), _ptr(w), _ptr(g_out), _ptr(dw),
                               _ptr(workspace), _nbytes(workspace), _stream(stream)), "fdnn_backward")


def link_desc(n_fft, n_data, users, antennas, taps, qam, pa, dpd=None) -> LinkDesc:
    d = dpd if dpd is not None else GmpDesc(0, 0, 0)
    return LinkDesc(int(n_fft), int(n_data), int(users), int(antennas), int(taps), int(qam), pa, d)


def zf_workspace_size(desc, n_ch) -> int:
    n = C.c_size_t(0)
    _check(lib().zf_workspace_size(C.byref(desc), int(n_ch), C.byref(n)), "zf_workspace_size")
    return n.value


def zf_precoder(desc, n_ch, h_est, p_total, all_bins, pt, alpha, workspace, stream=None):
    _check(lib().zf_precoder(C.byref(desc), int(n_ch), _ptr(h_est), float(p_total), int(bool(all_bins)), _ptr(pt),
                             _ptr(alpha), _ptr(workspace), _nbytes(workspace), _stream(stream)), "zf_precoder")


def ofdm_precode(desc, n_sym, sym_per_ch, pt, alpha, s, all_bins, x, stream=None):
    _check(lib().ofdm_precode(C.byref(desc), int(n_sym), int(sym_per_ch), _ptr(pt), _ptr(alpha), _ptr(s),
                              int(bool(all_bins)), _ptr(x), _stream(stream)), "ofdm_precode")


def link_workspace_size(desc, n_sym, sym_per_ch) -> int:
    n = C.c_size_t(0)
    _check(lib().link_workspace_size(C.byref(desc), int(n_sym), int(sym_per_ch), C.byref(n)),
           "link_workspace_size")
    return n.value


def ofdm_link(desc, n_sym, sym_per_ch, x, dpd_coef, pa_coef, g, h, alpha, noise, tx, r_out, errors, workspace,
              stream=None):
    g = complex(g)
    _check(lib().ofdm_link(C.byref(desc), int(n_sym), int(sym_per_ch), _ptr(x), _ptr(dpd_coef), _ptr(pa_coef),
                           g.real, g.imag, _ptr(h), _ptr(alpha), _ptr(noise), _ptr(tx), _ptr(r_out),
                           _ptr(errors), _ptr(workspace), _nbytes(workspace), _stream(stream)), "ofdm_link")


def ofdm_link_backward(desc, n_sym, sym_per_ch, x, pa_coef, g, h, alpha, g_r, g_x, workspace, stream=None):
    g = complex(g)
    _check(lib().ofdm_link_backward(C.byref(desc), int(n_sym), int(sym_per_ch), _ptr(x), _ptr(pa_coef), g.real,
                                    g.imag, _ptr(h), _ptr(alpha), _ptr(g_r), _ptr(g_x), _ptr(workspace),
                                    _nbytes(workspace), _stream(stream)), "ofdm_link_backward")


def ofdm_precode_backward(desc, n_sym, sym_per_ch, pt, alpha, g_x, all_bins, g_s, stream=None):
    _check(lib().ofdm_precode_backward(C.byref(desc), int(n_sym), int(sym_per_ch), _ptr(pt), _ptr(alpha), _ptr(g_x),
                                       int(bool(all_bins)), _ptr(g_s), _stream(stream)), "ofdm_precode_backward")


def dpd_acpr_workspace_size(n: int, nfft: int) -> int:
    return lib().dpd_acpr_workspace_size(n, nfft)


def cascade_acpr(y, n, nfft, half_bins, psd, acpr, workspace, stream=None):
    _check(lib().cascade_acpr(_ptr(y), n, nfft, half_bins, _ptr(psd), _ptr(acpr), _ptr(workspace),
                              workspace.numel() * workspace.element_size(), _stream(stream)),
           "cascade_acpr")


def dpd_profile_enable(on: bool = True):
    _check(lib().dpd_profile_enable(1 if on else 0), "dpd_profile_enable")


def dpd_profile_report() -> dict:
    """{kernel: (launches, total_ms)} since the last report; waits for the events."""
    buf = C.create_string_buffer(1 << 16)
    lib().dpd_profile_report(buf, len(buf))
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


def dpd_version() -> str:
    return lib().dpd_version().decode()
