"""GPU parity of the tuned path on TDNN shapes other than the paper's three sizes: the
generic instantiations (taps padded to 8, 16 or 32, width to 32, 64 or 128, 1..4 hidden
layers) against the FP64 oracle, forward, NMSE and gradient.  Among them the FD-NN-sized
core of Sec. V-A-1 (4 taps, one hidden layer of 15), degenerate sizes (1 tap, width 1)
and every padding bucket's edges."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import dpd_synth as S
from dpd_synth import Inputs
import gpu_helpers as H
import paper_2205_05158_amd as D

pytestmark = pytest.mark.gpu

# (taps, hidden layers, width)
SHAPES = [(4, 1, 15), (1, 1, 1), (3, 2, 7), (8, 3, 32), (11, 2, 50), (5, 4, 96), (17, 1, 100),
          (16, 4, 127), (20, 3, 64), (32, 4, 128)]
LENS = [5, 1000, 6001]


def announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)
    sys.stdout.flush()


def shape_inputs(T, nl, H_, per_stream=True, lens=LENS, seed=11):
    wl = dataclasses.replace(S.WORKLOADS["parity_16k"], name=f"generic_{T}_{nl}_{H_}", taps=T,
                             n_hidden=nl, hidden=H_, n_streams=len(lens), per_stream_params=per_stream)
    xs, ws, cs = [], [], []
    for s, n in enumerate(lens):
        xs.append(S.ofdm_signal(2048, 1200, -(-n // 2048), 64, np.random.default_rng(seed + s))[:n])
        ws.append(S.xavier_tdnn(T, nl, H_, 300 + s))
        cs.append(S.gmp_coefficients(wl.K, wl.M, wl.L, 400 + s))
    x = S.to_interleaved(np.concatenate(xs))
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    if per_stream:
        return Inputs(wl, x, off, np.stack(ws), np.stack(cs))
    return Inputs(wl, x, off, ws[0], cs[0])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "T%d_nl%d_H%d" % s)
def test_generic_shape_against_oracle(shape, prec):
    """Three ragged streams with their own parameter sets, residual DPD, complex gain."""
    T, nl, H_ = shape
    announce(f"generic TDNN shape T={T} nl={nl} H={H_} prec={prec}, streams {LENS}")
    inp = shape_inputs(T, nl, H_)
    g = 0.95 - 0.05j
    got = H.run_gpu(inp, precision=prec, residual=True, gain=g)
    ref = H.oracle_for(inp, residual=True, gain=g)
    H.check_cascade(inp, got, ref, prec)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fdnn_core_shared_parameters(prec):
    """The FD-NN-sized core (4 taps, one layer of 15) with one parameter set over
    frames, through the autograd boundary and a few Adam steps (the loss falls)."""
    announce(f"FD-NN-sized core T=4 nl=1 H=15, shared parameters, prec={prec}")
    inp = shape_inputs(4, 1, 15, per_stream=False, lens=[4096] * 4)
    got = H.run_gpu(inp, precision=prec)
    ref = H.oracle_for(inp)
    H.check_cascade(inp, got, ref, prec)
    cas = H.cascade_for(inp, precision=prec)
    x, c = H.to_dev(inp.x), H.to_dev(inp.coef)
    w = H.to_dev(inp.w).clone()
    losses, _ = cas.train(x, w, c, 50)
    torch.cuda.synchronize()
    first, last = float(losses[0, 0]), float(losses[-1, 0])
    print(f"  loss {first:.4e} -> {last:.4e} after 50 Adam steps", flush=True)
    assert last < first


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_padding_taps_masked(prec):
    """A NaN input sample reaches exactly the T outputs whose taps hold it, although the
    generic kernel for T = 4 computes features for 8 taps (the padding taps' features
    are masked, not only multiplied by zero weights)."""
    T, nl, H_ = 4, 1, 15
    announce(f"padding taps masked: NaN sample, T={T} nl={nl} H={H_} prec={prec}")
    inp = shape_inputs(T, nl, H_, per_stream=False, lens=[3000])
    n0 = 1234
    x_nan = inp.x.copy()
    x_nan[n0, 0] = np.nan
    cas = H.cascade_for(inp, precision=prec)
    u = cas.forward_u(H.to_dev(x_nan), H.to_dev(inp.w))
    torch.cuda.synchronize()
    u = u.cpu().numpy()
    bad = ~np.isfinite(u).all(axis=1)
    assert np.array_equal(np.flatnonzero(bad), np.arange(n0, n0 + T))
    # elsewhere the outputs are those of the input without the NaN sample (zero there)
    x0 = inp.x.copy()
    x0[n0] = 0.0
    ref = H.oracle_for(Inputs(inp.workload, x0, inp.offsets, inp.w, inp.coef), grad=False)
    keep = ~bad
    err = H.per_sample_rel(u[keep], ref.u[keep])
    assert err <= (H.FP32_SAMPLE if prec == "fp32" else H.BF16_SAMPLE)


def test_exact_and_generic_dispatch():
    """The paper's three sizes run on their own kernels, neighbouring sizes on generic
    instantiations; both report a launch shape."""
    b = D.make_batch([0, 1000])
    g = D.gmp_desc(5, 3, 2)
    for shape in [(4, 2, 20), (4, 2, 21), (10, 3, 64), (10, 3, 63), (16, 4, 128), (16, 4, 127)]:
        for prec in ("fp32", "bf16"):
            assert D.dpd_tune_get(D.tdnn_desc(*shape, precision=prec), g, b)["fwd_waves"] in (8, 12)


# GMP orders without an instantiation of their own (run on the zero-padded (9, 7, 4)
# kernels): the degenerate linear PA (K 1, no memory), memory only, cross terms only at
# the padded bound, and mixed orders
GMP_ORDERS = [(1, 0, 0), (3, 2, 1), (6, 4, 2), (9, 0, 4), (2, 7, 0), (8, 6, 3)]


def gmp_order_inputs(K, M, L, lens=LENS):
    wl = dataclasses.replace(S.WORKLOADS["parity_16k"], name=f"gmp_{K}_{M}_{L}", K=K, M=M, L=L,
                             n_streams=len(lens), per_stream_params=True)
    xs, ws, cs = [], [], []
    for s, n in enumerate(lens):
        xs.append(S.ofdm_signal(2048, 1200, -(-n // 2048), 64, np.random.default_rng(21 + s))[:n])
        ws.append(S.xavier_tdnn(wl.taps, wl.n_hidden, wl.hidden, 500 + s))
        cs.append(S.gmp_coefficients(K, M, L, 600 + s))
    x = S.to_interleaved(np.concatenate(xs))
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return Inputs(wl, x, off, np.stack(ws), np.stack(cs))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("order", GMP_ORDERS, ids=lambda o: "K%d_M%d_L%d" % o)
def test_padded_gmp_order_against_oracle(order, prec):
    """The cascade and its gradient with GMP orders that run on the zero-padded kernels,
    three ragged streams with their own parameter sets, against the FP64 oracle; and the
    forward-only cascade, whose GMP forward kernel pads the same way."""
    K, M, L = order
    announce(f"padded GMP order K={K} M={M} L={L} prec={prec}, streams {LENS}")
    inp = gmp_order_inputs(K, M, L)
    got = H.run_gpu(inp, precision=prec)
    ref = H.oracle_for(inp)
    H.check_cascade(inp, got, ref, prec)
    fwd = H.run_gpu(inp, precision=prec, grad=False)
    H.check_cascade(inp, fwd, ref, prec, grad=False)


def test_padded_gmp_order_autotuned():
    """The autotuner takes a GMP order without kernels of its own (it times the padded
    kernels); the cascade at the picked shapes against the FP64 oracle."""
    announce(f"padded GMP order (6, 4, 2) autotuned, streams {LENS}")
    inp = gmp_order_inputs(6, 4, 2)
    cas = H.cascade_for(inp, precision="bf16")
    x, w, c = H.to_dev(inp.x), H.to_dev(inp.w), H.to_dev(inp.coef)
    try:
        pick = cas.autotune(x, w, c, reps=1)
        print(f"  picked {pick}", flush=True)
        out = cas.run(x, w, c)
        torch.cuda.synchronize()
        got = {k: (None if v is None else v.cpu().numpy()) for k, v in out.items()}
    finally:
        cas.set_tune(None)
    H.check_cascade(inp, got, H.oracle_for(inp), "bf16")
