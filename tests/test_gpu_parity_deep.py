"""Parity of the hot path against the FP64 oracle where it is hardest to meet:
the BF16 gradient of the 16-tap 4x128 model on 2^20 samples (every reverse-mode
workgroup accumulating dozens of tiles, in both backward grids the autotuner chooses
from) and on 2^22 samples at the autotuned shape, the FP32 forward NMSE of the whole 2^22-sample workload, and the cascade at a
trained operating point (Sec. V-A-2: the DPD trained by MSE through the chain to a low
error), where the NMSE criterion is tightest.  Reported besides the criteria: the
output-parity NMSE 10 log10(sum |y_gpu - y_64|^2 / sum |y_64|^2)."""
import sys

import numpy as np
import pytest
import torch

import dpd_synth as S
import gpu_helpers as H
import oracle as O

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bf16_slice():
    """The first 2^20 samples of the bf16_16m workload and their oracle cascade."""
    inp = S.make_workload("bf16_16m", max_len=1 << 20)
    return inp, H.oracle_for(inp)


@pytest.mark.parametrize("bwd_per_cu", [1, 2])
def test_bf16_gradient_2p20_against_oracle(bf16_slice, bwd_per_cu):
    inp, ref = bf16_slice
    announce(f"bf16_16m first 2^20 samples, BF16 gradient vs oracle, bwd_wg_per_cu={bwd_per_cu}")
    cas = H.cascade_for(inp)
    shape = dict(cas.tune(), bwd_wg_per_cu=bwd_per_cu)
    cas.set_tune(shape)
    tiles = (inp.n_total + 63) // 64
    grid = min(tiles, bwd_per_cu * torch.cuda.get_device_properties(0).multi_processor_count)
    assert tiles // grid >= 16, "every reverse-mode workgroup accumulates >= 16 tiles"
    x, w, c = H.to_dev(inp.x), H.to_dev(inp.w), H.to_dev(inp.coef)
    out = cas.run(x, w, c)
    torch.cuda.synchronize()
    got = {k: (None if v is None else v.cpu().numpy()) for k, v in out.items()}
    cas.set_tune(None)
    wl = inp.workload
    per_tensor = H.grad_rel_per_tensor(got["dw"], ref.dw.reshape(got["dw"].shape), wl.taps, wl.n_hidden,
                                       wl.hidden)
    op = H.output_parity_db(got["y"], ref.y)
    print(f"  {tiles // grid} tiles per workgroup; per-tensor gradient rel err "
          + ", ".join(f"{k} {v:.1e}" for k, v in per_tensor.items()) + f"; output parity {op:.1f} dB",
          flush=True)
    H.check_cascade(inp, got, ref, "bf16")
    assert max(per_tensor.values()) <= H.BF16_GRAD_LARGE
    assert op <= H.BF16_OUTPUT_PARITY_DB


def test_bf16_gradient_2p22_against_oracle():
    """A quarter of the bf16_16m workload (its first 2^22 samples) at the bench's
    autotuned launch shape: the BF16 gradient per tensor, the NMSE and the output parity
    against the oracle's cascade on the whole slice (every reverse-mode workgroup
    accumulating about 64 tiles)."""
    announce("bf16_16m first 2^22 samples, BF16 gradient vs oracle at the autotuned shape")
    inp = S.make_workload("bf16_16m", max_len=1 << 22)
    cas = H.cascade_for(inp)
    x, w, c = H.to_dev(inp.x), H.to_dev(inp.w), H.to_dev(inp.coef)
    cas.autotune(x, w, c, reps=2)
    out = cas.run(x, w, c)
    torch.cuda.synchronize()
    got = {k: (None if v is None else v.cpu().numpy()) for k, v in out.items()}
    cas.set_tune(None)
    del x, w, c, out
    ref = H.oracle_for(inp)
    wl = inp.workload
    per_tensor = H.grad_rel_per_tensor(got["dw"], ref.dw.reshape(got["dw"].shape), wl.taps, wl.n_hidden,
                                       wl.hidden)
    op = H.output_parity_db(got["y"], ref.y)
    print("  per-tensor gradient rel err " + ", ".join(f"{k} {v:.1e}" for k, v in per_tensor.items())
          + f"; output parity {op:.1f} dB", flush=True)
    H.check_cascade(inp, got, ref, "bf16")
    assert max(per_tensor.values()) <= H.BF16_GRAD_LARGE
    assert op <= H.BF16_OUTPUT_PARITY_DB


def test_fwd_4m_full_size_against_oracle():
    """The whole 2^22-sample FP32 forward workload: every sample of u and y and the NMSE
    against the oracle's."""
    announce("fwd_4m: 2^22 samples, FP32 forward vs oracle on every sample")
    inp = S.make_workload("fwd_4m")
    got = H.run_gpu(inp, grad=False)
    ref = H.oracle_for(inp, grad=False)
    op = H.output_parity_db(got["y"], ref.y)
    print(f"  output parity {op:.1f} dB", flush=True)
    H.check_cascade(inp, got, ref, "fp32", grad=False)
    assert op <= H.FP32_OUTPUT_PARITY_DB


TRAINED = {
    # workload, slice, precision, Adam steps, NMSE (dB) the device run must reach
    "fp32": ("train_1m_8f", None, "fp32", 2000, -20.0),
    "bf16": ("bf16_16m", 1 << 20, "bf16", 400, -12.0),
}


@pytest.mark.parametrize("which", ["fp32", "bf16"])
def test_trained_operating_point(which):
    """Direct learning on the device (dpd_backward + Adam, learning rate 0.001) to a low
    NMSE, then the cascade at the trained weights against the oracle: NMSE gap, output
    parity, per-sample error of u and y, and the gradient."""
    name, max_len, prec, steps, target_db = TRAINED[which]
    announce(f"trained operating point: {name} slice {max_len} {prec}, {steps} Adam steps")
    inp = S.make_workload(name, max_len=max_len)
    cas = H.cascade_for(inp, precision=prec)
    x, c = H.to_dev(inp.x), H.to_dev(inp.coef)
    w = H.to_dev(inp.w).clone()
    losses, _ = cas.train(x, w, c, steps)
    torch.cuda.synchronize()
    trained = S.Inputs(inp.workload, inp.x, inp.offsets, w.cpu().numpy(), inp.coef)
    got = H.run_gpu(trained, precision=prec)
    nmse_db = float(got["nmse"][-1, 2])
    print(f"  NMSE {10 * np.log10(losses[0, 0].item()):.2f} dB -> {nmse_db:.2f} dB after {steps} steps",
          flush=True)
    assert nmse_db <= target_db
    ref = H.oracle_for(trained)
    wl = inp.workload
    op = H.output_parity_db(got["y"], ref.y)
    per_tensor = H.grad_rel_per_tensor(got["dw"], ref.dw.reshape(got["dw"].shape), wl.taps, wl.n_hidden,
                                       wl.hidden)
    gap = abs(nmse_db - H.db(ref.E.sum() / ref.R.sum()))
    print(f"  NMSE gap {gap:.2e} dB; output parity {op:.1f} dB; gradient rel err (worst tensor) "
          f"{max(per_tensor.values()):.2e}", flush=True)
    H.check_cascade(trained, got, ref, prec, grad=False)
    assert op <= (H.FP32_OUTPUT_PARITY_DB if prec == "fp32" else H.BF16_OUTPUT_PARITY_DB)
    if prec == "fp32":
        assert max(per_tensor.values()) <= H.FP32_GRAD
