"""Direct-learning training on the device (dpd_backward + dpd_adam_step) against the
FP64 oracle of oracle/adam.py: the Adam kernel alone on ragged lengths and gradient
scales, and whole training runs (loss trajectory and weights)."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import oracle.adam as OA
import dpd_synth as S
import paper_2205_05158_amd as D
import gpu_helpers as H

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n", [1, 3, 4, 1027, 60162])
def test_adam_kernel_matches_oracle(n):
    """Five steps with fresh gradients of mixed scale and sign; float32 on the device
    against float64 from the same float32 inputs.  Bound: each step rounds w once
    (2^-24 |w|) and the update to a few ulps (lr x 1e-6); the moments to float32
    rounding of each of their terms."""
    announce(f"adam kernel n={n}")
    rng = np.random.default_rng(n)
    w0 = rng.standard_normal(n).astype(np.float32)
    grads = [(rng.standard_normal(n) * 10.0 ** rng.uniform(-6, 1, n)).astype(np.float32)
             for _ in range(5)]
    w = H.to_dev(w0)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    wr, mr, vr = w0.astype(np.float64), np.zeros(n), np.zeros(n)
    for t, g in enumerate(grads, start=1):
        D.dpd_adam_step(H.to_dev(g), w, m, v, t)
        wr, mr, vr = OA.adam_step(wr, mr, vr, g.astype(np.float64), t)
    torch.cuda.synchronize()
    steps = len(grads)
    np.testing.assert_allclose(w.cpu().numpy(), wr, rtol=steps * 1.2e-7, atol=steps * 2e-9)
    # the moments are sums of signed terms (the first one cancels): bound their error by
    # float32 rounding of each term, including of the rounded constants 1 - beta
    s1 = sum(0.1 * 0.9 ** (steps - t) * np.abs(g.astype(np.float64)) for t, g in enumerate(grads, 1))
    s2 = sum(1e-3 * 0.999 ** (steps - t) * g.astype(np.float64) ** 2 for t, g in enumerate(grads, 1))
    assert np.all(np.abs(m.cpu().numpy() - mr) <= 1e-6 * s1)
    assert np.all(np.abs(v.cpu().numpy() - vr) <= 1e-6 * s2)


@pytest.mark.parametrize("workload,kw,prec,steps", [
    ("parity_16k", {}, "fp32", 8),
    ("batched_64s", dict(n_streams=3, max_len=5000), "fp32", 6),
    ("bf16_16m", dict(max_len=8000), "bf16", 4),
])
def test_training_run_matches_oracle(workload, kw, prec, steps):
    """A few direct-learning steps (learning rate 0.001): the loss before every step
    within the path's NMSE tolerance of the oracle's run, and the total weight change
    within 1 % (fp32) / 5 % (bf16) of the oracle's in L2 norm per parameter set."""
    announce(f"training {workload} {kw} prec={prec} steps={steps}")
    inp = S.make_workload(workload, **kw)
    wl = inp.workload
    model = O.Model(wl.taps, wl.n_hidden, wl.hidden, wl.K, wl.M, wl.L)
    ref_losses, ref_w = OA.train(inp.x, inp.offsets, inp.w, inp.coef, model, steps,
                                 per_stream=wl.per_stream_params)
    cas = H.cascade_for(inp, precision=prec)
    x, w, c = H.to_dev(inp.x), H.to_dev(inp.w), H.to_dev(inp.coef)
    losses, (m, v, t) = cas.train(x, w, c, steps)
    torch.cuda.synchronize()
    assert t == steps
    got = losses.cpu().numpy()
    tol_db = H.FP32_NMSE_DB if prec == "fp32" else H.BF16_NMSE_DB
    gap = np.abs(10 * np.log10(got) - 10 * np.log10(ref_losses.reshape(got.shape)))
    print(f"  loss dB first {10 * np.log10(got[0])} last {10 * np.log10(got[-1])}; max gap {gap.max():.2e}",
          flush=True)
    assert gap.max() <= tol_db
    dw_got = w.cpu().numpy().reshape(-1, cas.P) - inp.w.reshape(-1, cas.P)
    dw_ref = ref_w.reshape(-1, cas.P) - inp.w.reshape(-1, cas.P)
    rel = np.linalg.norm(dw_got - dw_ref, axis=1) / np.linalg.norm(dw_ref, axis=1)
    print(f"  weight-change rel err per set max {rel.max():.2e}", flush=True)
    assert rel.max() <= (1e-2 if prec == "fp32" else 5e-2)
