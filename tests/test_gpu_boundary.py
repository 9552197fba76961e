"""GPU checks of the boundary's status reporting and of the loss arithmetic the library
does for its callers: non-finite samples counted in the NMSE records (Sec. II-B target)
without affecting other streams or parameter sets, the library-computed loss used by the
autograd boundary, and the symbol MSE of the receiver-side criterion (Sec. V-A-2)
against the oracle's."""
import sys

import numpy as np
import pytest
import torch

import dpd_synth as S
import gpu_helpers as H
import oracle as O
import oracle.fdcnn as OF
import paper_2205_05158_amd as D
from dpd_synth import Inputs

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)
    sys.stdout.flush()


def _oracle_nonfinite(inp, ref, G=1.0):
    """Per-stream count of samples whose |y - G x|^2 or |G x|^2 is not finite (FP64)."""
    x = H.cplx(inp.x)
    with np.errstate(all="ignore"):
        gx = G * x
        e2 = np.abs(ref.y - gx) ** 2 + np.abs(gx) ** 2
        bad = ~np.isfinite(e2)
    off = inp.offsets
    return [int(bad[off[s]:off[s + 1]].sum()) for s in range(len(off) - 1)]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_nonfinite_samples_counted_and_contained(prec):
    """NaN samples in stream 1 and an infinite sample in stream 2 of a four-stream batch
    with per-stream parameters: the records of those streams count exactly the samples
    the FP64 oracle finds non-finite, dpd_nmse_status reports DPD_ERR_NONFINITE, their
    sets' loss is not finite, and streams 0 and 3 (records, loss, dW) are bitwise the
    same as in the clean run."""
    announce(f"non-finite samples, 4 streams, prec={prec}")
    clean = S.make_workload("batched_64s", n_streams=4, max_len=5000)
    x = clean.x.copy()
    off = clean.offsets
    x[off[1] + 100] = np.nan
    x[off[1] + 2001, 1] = np.nan
    x[off[2] + 37, 0] = np.inf
    bad = Inputs(clean.workload, x, off, clean.w, clean.coef)
    got0 = H.run_gpu(clean, precision=prec)
    got = H.run_gpu(bad, precision=prec)
    assert D.dpd_nmse_status(got0["nmse"]) == D.DPD_OK
    assert D.dpd_nmse_status(got["nmse"]) == D.DPD_ERR_NONFINITE
    with np.errstate(all="ignore"):
        ref = H.oracle_for(bad, grad=False)
    want = _oracle_nonfinite(bad, ref)
    counts = [int(v) for v in got["nmse"][:-1, 3]]
    print(f"  non-finite counts gpu {counts} oracle {want}", flush=True)
    assert counts == want
    assert want[1] > 0 and want[2] > 0 and want[0] == 0 and want[3] == 0
    assert int(got["nmse"][-1, 3]) == sum(want)
    assert np.all(got0["nmse"][:, 3] == 0)
    for s in (1, 2):
        assert not np.isfinite(got["loss"][s])
        assert not np.all(np.isfinite(got["dw"][s]))
    for s in (0, 3):
        np.testing.assert_array_equal(got["nmse"][s], got0["nmse"][s])
        np.testing.assert_array_equal(got["loss"][s], got0["loss"][s])
        np.testing.assert_array_equal(got["dw"][s], got0["dw"][s])


def test_nonfinite_forward_only_records():
    """The forward-only path (cascade_nmse on given y) counts the same samples."""
    announce("non-finite samples, cascade_nmse")
    inp = S.make_workload("parity_16k")
    cas = H.cascade_for(inp)
    x = H.to_dev(inp.x)
    out = cas.run(x, H.to_dev(inp.w), H.to_dev(inp.coef), want_grad=False)
    y = out["y"].clone()
    y[10, 0] = float("nan")
    y[11, 1] = float("inf")
    y[5000] = float("-inf")
    nm = cas.nmse(y, x).cpu().numpy()
    assert int(nm[0, 3]) == 3 and int(nm[-1, 3]) == 3
    assert D.dpd_nmse_status(nm) == D.DPD_ERR_NONFINITE
    nm0 = cas.nmse(out["y"], x).cpu().numpy()
    assert int(nm0[0, 3]) == 0 and D.dpd_nmse_status(nm0) == D.DPD_OK


def test_autograd_forward_uses_library_loss():
    """CascadeFn without a weight gradient returns the library's pooled loss, equal to
    the oracle's loss and to the reverse-mode call's loss up to float32 summation order."""
    announce("CascadeFn no-grad loss")
    inp = S.make_workload("batched_64s", n_streams=3, max_len=7000)
    cas = H.cascade_for(inp)
    x, w, c = H.to_dev(inp.x), H.to_dev(inp.w), H.to_dev(inp.coef)
    with torch.no_grad():
        l_fwd = D.CascadeFn.apply(w, x, c, cas).cpu().numpy()
    l_bwd = cas.backward(x, w, c)[0].cpu().numpy()
    ref = H.oracle_for(inp, grad=False)
    np.testing.assert_allclose(l_fwd, ref.E / ref.R, rtol=1e-5)
    np.testing.assert_allclose(l_fwd, l_bwd, rtol=1e-5)


@pytest.mark.parametrize("n", [1, 3, 4095, 4096, 4097, 100003])
def test_symbol_mse_against_oracle(n):
    """dpd_symbol_mse: loss and gradient seed against the oracle's MSE of Sec. V-A-2."""
    announce(f"symbol MSE n={n}")
    rng = np.random.default_rng(n)
    z = rng.standard_normal((n, 2)).astype(np.float32)
    t = rng.standard_normal((n, 2)).astype(np.float32)
    out = torch.empty(2, dtype=torch.float32, device="cuda")
    grad = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    ws = torch.empty(D.dpd_symbol_mse_workspace_size(n), dtype=torch.uint8, device="cuda")
    D.dpd_symbol_mse(n, H.to_dev(z), H.to_dev(t), out, grad, ws)
    torch.cuda.synchronize()
    loss_ref, g_ref = OF.mse_to_target(H.cplx(z), H.cplx(t))
    o = out.cpu().numpy()
    assert o[1] == 0
    np.testing.assert_allclose(o[0], loss_ref, rtol=2e-6)
    np.testing.assert_allclose(H.cplx(grad.cpu().numpy()), g_ref, rtol=2e-7, atol=1e-7 * np.abs(g_ref).max())
    # a NaN value is counted and makes the loss non-finite; no gradient requested
    z[n // 2, 0] = np.nan
    D.dpd_symbol_mse(n, H.to_dev(z), H.to_dev(t), out, None, ws)
    o = out.cpu().numpy()
    assert o[1] == 1 and not np.isfinite(o[0])
