"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Sizes here let the oracle finish in seconds while spanning
many tiles, several streams and ragged tails; the full workload sizes are covered
in test_gpu_fullsize.py."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import dpd_synth as S
from dpd_synth import Inputs, Workload
import gpu_helpers as H

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)
    sys.stdout.flush()


check_cascade = H.check_cascade


@pytest.mark.parametrize("impl,prec", [("tuned", "fp32"), ("plain", "fp32"), ("tuned", "bf16")])
def test_parity_16k(impl, prec):
    announce(f"parity_16k impl={impl} prec={prec}")
    inp = S.make_workload("parity_16k")
    got = H.run_gpu(inp, precision=prec, impl=impl)
    ref = H.oracle_for(inp)
    check_cascade(inp, got, ref, prec)


def _ragged_inputs(per_stream, lens, seed=5):
    wl = S.WORKLOADS["batched_64s" if per_stream else "train_1m_8f"]
    xs, ws, cs = [], [], []
    for s, n in enumerate(lens):
        sig = S.ofdm_signal(4096, 1024, -(-n // 4096), 64, np.random.default_rng(seed + s))[:n]
        xs.append(sig)
        ws.append(S.xavier_tdnn(wl.taps, wl.n_hidden, wl.hidden, 100 + s))
        cs.append(S.gmp_coefficients(wl.K, wl.M, wl.L, 200 + s))
    x = S.to_interleaved(np.concatenate(xs))
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    if per_stream:
        return Inputs(wl, x, off, np.stack(ws), np.stack(cs))
    return Inputs(wl, x, off, ws[0], cs[0])


RAGGED = [1, 3, 127, 128, 129, 1000, 4097]


@pytest.mark.parametrize("impl", ["tuned", "plain"])
@pytest.mark.parametrize("per_stream", [True, False])
def test_ragged_streams(impl, per_stream):
    """Streams shorter than the tap window and the GMP memory, exact tile multiples and
    ragged tails; per-stream or shared parameter sets; complex gain; residual DPD."""
    announce(f"ragged streams {RAGGED} impl={impl} per_stream={per_stream}")
    inp = _ragged_inputs(per_stream, RAGGED)
    g = 0.9 + 0.1j
    got = H.run_gpu(inp, precision="fp32", impl=impl, residual=True, gain=g)
    ref = H.oracle_for(inp, residual=True, gain=g)
    check_cascade(inp, got, ref, "fp32")


@pytest.mark.parametrize("impl", ["tuned", "plain"])
def test_frames_shared_parameters(impl):
    """8 zero-padded frames sharing one parameter set, pooled loss (frames shortened)."""
    announce(f"train_1m_8f frames of 6000 impl={impl}")
    inp = S.make_workload("train_1m_8f", max_len=6000)
    got = H.run_gpu(inp, precision="fp32", impl=impl)
    ref = H.oracle_for(inp)
    check_cascade(inp, got, ref, "fp32")


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_large_model_shortened(prec):
    """The 16-tap, 4x128 TDNN with GMP (9, 7, 4) on a 20000-sample PAPR-clipped slice."""
    announce(f"bf16_16m model, 20000 samples, prec={prec}")
    inp = S.make_workload("bf16_16m", max_len=20000)
    got = H.run_gpu(inp, precision=prec)
    ref = H.oracle_for(inp)
    check_cascade(inp, got, ref, prec)


def test_batched_streams_subset():
    """First 6 streams of the 64-stream batch (own parameters each), shortened."""
    announce("batched_64s first 6 streams <= 9000 samples")
    inp = S.make_workload("batched_64s", n_streams=6, max_len=9000)
    got = H.run_gpu(inp)
    ref = H.oracle_for(inp)
    check_cascade(inp, got, ref, "fp32")


def test_zero_dpd_output_gradient_is_finite():
    """u = 0 exactly on a stretch (zero input, residual DPD with zero output layer):
    the |u| derivative uses the value 0 there, as the oracle does."""
    announce("u == 0 stretch")
    inp = S.make_workload("parity_16k")
    wl = inp.workload
    x = inp.x.copy()
    x[100:400] = 0.0
    w = inp.w.copy()
    layers = O.unpack_tdnn(w.astype(np.float64), wl.taps, wl.n_hidden, wl.hidden)
    n_out = 2 * wl.hidden + 2
    w[-n_out:] = 0.0
    inp2 = Inputs(wl, x, inp.offsets, w, inp.coef)
    got = H.run_gpu(inp2, residual=True)
    ref = H.oracle_for(inp2, residual=True)
    assert np.all(np.isfinite(got["dw"]))
    assert np.all(got["u"][150:350] == 0.0)
    check_cascade(inp2, got, ref, "fp32")
    del layers


def test_determinism_bitwise():
    announce("determinism: two identical calls")
    inp = S.make_workload("batched_64s", n_streams=5, max_len=30000)
    a = H.run_gpu(inp)
    b = H.run_gpu(inp)
    for k in ("u", "y", "nmse", "dw", "loss"):
        assert np.array_equal(a[k], b[k]), k


def test_separate_calls_match_cascade():
    """dpd_forward + pa_gmp_forward + cascade_nmse give what dpd_cascade gives."""
    announce("separate ABI calls vs dpd_cascade")
    inp = S.make_workload("parity_16k")
    cas = H.cascade_for(inp)
    x, w, c = H.to_dev(inp.x), H.to_dev(inp.w), H.to_dev(inp.coef)
    u = cas.forward_u(x, w)
    y = cas.pa(u, c)
    nm = cas.nmse(y, x)
    full = cas.run(x, w, c)
    torch.cuda.synchronize()
    assert torch.equal(u, full["u"]) and torch.equal(y, full["y"])
    np.testing.assert_allclose(nm.cpu().numpy(), full["nmse"].cpu().numpy(), rtol=1e-6)


def test_autograd_function():
    announce("CascadeFn autograd")
    import paper_2205_05158_amd as D
    inp = S.make_workload("parity_16k")
    cas = H.cascade_for(inp)
    x, c = H.to_dev(inp.x), H.to_dev(inp.coef)
    w = H.to_dev(inp.w).requires_grad_(True)
    loss = D.CascadeFn.apply(w, x, c, cas)
    (3.0 * loss.sum()).backward()
    ref_loss, ref_dw = cas.backward(x, w.detach(), c)
    torch.cuda.synchronize()
    assert torch.allclose(loss.detach(), ref_loss)
    assert torch.allclose(w.grad, 3.0 * ref_dw)
    with torch.no_grad():
        l2 = D.CascadeFn.apply(w.detach(), x, c, cas)
    assert torch.allclose(l2, ref_loss, rtol=1e-5)


def test_acpr_matches_oracle_psd():
    """PSD/ACPR of the GPU's PA output against the oracle's PSD of the oracle's own
    PA output on the same 2^18-sample input."""
    announce("Welch PSD / ACPR on a 2^18-sample PA output")
    import paper_2205_05158_amd as D
    inp = S.make_workload("fwd_4m", max_len=1 << 18)
    got = H.run_gpu(inp, grad=False)
    ref = H.oracle_for(inp, grad=False)
    y = got["y"]
    n = y.shape[0]
    ws = torch.empty(D.dpd_acpr_workspace_size(n, 4096), dtype=torch.uint8, device="cuda")
    psd = torch.empty(4096, dtype=torch.float32, device="cuda")
    acpr = torch.empty(3, dtype=torch.float32, device="cuda")
    D.cascade_acpr(H.to_dev(y), n, 4096, 512, psd, acpr, ws)
    torch.cuda.synchronize()
    ref_psd = O.welch_psd(ref.y, 4096)
    np.testing.assert_allclose(psd.cpu().numpy(), ref_psd, rtol=2e-4, atol=1e-7 * ref_psd.max())
    ref_acpr = O.acpr_db(ref_psd, 512)
    print(f"  ACPR gpu {acpr.cpu().numpy()} oracle {ref_acpr}", flush=True)
    assert np.max(np.abs(acpr.cpu().numpy() - np.array(ref_acpr))) < 0.01


@pytest.mark.parametrize("nfft", [256, 1024, 4096])
def test_welch_sizes_against_oracle(nfft):
    """Welch PSD and ACPR of one PA output at every transform path: the radix-16
    4096-point kernel and the in-LDS radix-2 kernel of the other sizes."""
    announce(f"Welch PSD nfft={nfft} on a 2^16-sample PA output")
    import paper_2205_05158_amd as D
    inp = S.make_workload("fwd_4m", max_len=1 << 16)
    ref = H.oracle_for(inp, grad=False)
    y = np.stack([ref.y.real, ref.y.imag], -1).astype(np.float32)
    n = y.shape[0]
    hb = nfft // 8 - 1
    ws = torch.empty(D.dpd_acpr_workspace_size(n, nfft), dtype=torch.uint8, device="cuda")
    psd = torch.empty(nfft, dtype=torch.float32, device="cuda")
    acpr = torch.empty(3, dtype=torch.float32, device="cuda")
    D.cascade_acpr(H.to_dev(y), n, nfft, hb, psd, acpr, ws)
    torch.cuda.synchronize()
    ref_psd = O.welch_psd(y[:, 0].astype(np.float64) + 1j * y[:, 1], nfft)
    np.testing.assert_allclose(psd.cpu().numpy(), ref_psd, rtol=2e-4, atol=1e-7 * ref_psd.max())
    ref_acpr = np.array(O.acpr_db(ref_psd, hb))
    assert np.max(np.abs(acpr.cpu().numpy() - ref_acpr)) < 0.01
