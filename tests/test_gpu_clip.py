"""GPU parity of the ideal linear-clipping PA (Sec. V-B-2) and of the cascade DPD ->
clipping PA -> NMSE with its gradient, through the C ABI, against the FP64 oracle
(oracle/clip_pa.py) on the same seeded inputs."""
import sys

import numpy as np
import pytest
import torch

import dpd_synth as S
from dpd_synth import Inputs
import gpu_helpers as H
import oracle as O
import paper_2205_05158_amd as D
from test_gpu_generic_shapes import shape_inputs

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)
    sys.stdout.flush()


def test_pa_clip_forward_elementwise():
    """Random samples on both sides of the clip, exact zeros, samples exactly at the clip
    level, huge finite samples (whose squared magnitude overflows float32), a NaN."""
    announce("pa_clip_forward elementwise")
    rng = np.random.default_rng(7)
    n = 100003
    u = ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) * 1.2).astype(np.complex64)
    A = np.float32(1.25)
    u[:5] = 0
    u[5:9] = [A, -A, 1j * A, -1j * A]
    u[9:12] = [3e30 + 4e30j, -1e38, 2e19 - 2e19j]
    u[12] = np.nan
    uil = np.stack([u.real, u.imag], -1).astype(np.float32)
    ud = H.to_dev(uil)
    y = torch.empty_like(ud)
    D.pa_clip_forward(n, ud, float(A), y)
    inplace = ud.clone()
    D.pa_clip_forward(n, inplace, float(A), inplace)
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    assert np.array_equal(got, inplace.cpu().numpy(), equal_nan=True)
    u64 = uil[:, 0].astype(np.float64) + 1j * uil[:, 1]
    ref = O.clip_forward(u64, float(A))
    g = got[:, 0].astype(np.float64) + 1j * got[:, 1]
    assert np.isnan(g[12]) and np.isfinite(g[np.arange(n) != 12]).all()
    keep = np.arange(n) != 12
    err = np.abs(g[keep] - ref[keep]) / np.maximum(np.abs(ref[keep]), 1.0)
    print(f"  max rel err {err.max():.2e}", flush=True)
    assert err.max() <= 1e-6
    # below the clip the PA is the identity, bit for bit
    below = np.abs(u64) <= A
    assert np.array_equal(got[below], uil[below])


def _clip_level(inp, ref_u, frac=0.1):
    """A clipping level with about frac of the oracle's |u| above it, kept at least 1e-5
    (relative) away from every |u| so that the float32 and float64 sides take the same
    branch for every sample."""
    r = np.sort(np.abs(ref_u))
    k = int((1 - frac) * r.size)
    A = float(0.5 * (r[k] + r[k + 1]))
    assert np.min(np.abs(r - A)) > 1e-5 * A
    return A


CASES = [("tuned", "fp32", (10, 3, 64)), ("tuned", "bf16", (16, 4, 128)), ("plain", "fp32", (4, 2, 20)),
         ("tuned", "fp32", (4, 1, 15)), ("tuned", "bf16", (4, 1, 15))]


@pytest.mark.parametrize("impl,prec,shape", CASES, ids=lambda v: str(v))
def test_clip_cascade_against_oracle(impl, prec, shape):
    """Ragged streams with their own parameter sets, residual DPD, complex gain, about
    10 % of the samples clipped: u, y, NMSE per stream and pooled, loss and gradient."""
    T, nl, H_ = shape
    announce(f"clip cascade impl={impl} prec={prec} T={T} nl={nl} H={H_}")
    inp = shape_inputs(T, nl, H_, lens=[7, 1500, 9001])
    model = O.Model(T, nl, H_, 1, 0, 0, True)
    g = 0.95 - 0.05j
    probe = O.cascade_clip(inp.x, inp.offsets, inp.w, model, 1e30, G=g, per_stream=True, grad=False)
    A = _clip_level(inp, probe.u)
    ref = O.cascade_clip(inp.x, inp.offsets, inp.w, model, A, G=g, per_stream=True)
    cas = D.ClipCascade(T, nl, H_, inp.offsets, A, per_stream_params=True, residual=True, precision=prec,
                        impl=impl, gain=g)
    out = cas.run(H.to_dev(inp.x), H.to_dev(inp.w))
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    clipped = float(np.mean(np.abs(ref.y - ref.u) > 0))
    print(f"  clip level {A:.4f}, {100 * clipped:.1f} % of samples clipped", flush=True)
    assert 0.05 < clipped < 0.2
    H.check_cascade(inp, got, ref, prec)


def test_clip_cascade_forward_only_matches_full():
    """Without dw the call gives the same u, y and records (bitwise)."""
    announce("clip cascade forward-only vs with gradient")
    inp = shape_inputs(10, 3, 64, lens=[3000, 2000])
    cas = D.ClipCascade(10, 3, 64, inp.offsets, 1.3, per_stream_params=True, residual=True)
    x, w = H.to_dev(inp.x), H.to_dev(inp.w)
    a = cas.run(x, w)
    b = cas.run(x, w, want_grad=False)
    torch.cuda.synchronize()
    for k in ("u", "y", "nmse"):
        assert torch.equal(a[k], b[k]), k


def test_clip_pa_of_unclipped_cascade_is_identity():
    """A clipping level above every |u|: y == u exactly, and the cascade's loss and
    gradient equal those of the GMP cascade with the unit-gain PA (K = 1, M = L = 0,
    a_00 = 1; the plain kernels, which take every GMP order) to float32 rounding."""
    announce("clip cascade without clipping vs unit-gain GMP cascade")
    inp = S.make_workload("parity_16k")
    wl = inp.workload
    x, w = H.to_dev(inp.x), H.to_dev(inp.w)
    out = {}
    for impl in ("tuned", "plain"):
        cas = D.ClipCascade(wl.taps, wl.n_hidden, wl.hidden, inp.offsets, 1e30, impl=impl)
        out[impl] = cas.run(x, w)
    gcas = D.Cascade(wl.taps, wl.n_hidden, wl.hidden, 1, 0, 0, inp.offsets, impl="plain")
    coef = torch.tensor([[1.0, 0.0]], device="cuda")
    ref = gcas.run(x, w, coef)
    torch.cuda.synchronize()
    for impl, o in out.items():
        assert torch.equal(o["y"], o["u"]), impl
        assert torch.allclose(o["u"], ref["u"], rtol=1e-5, atol=1e-6), impl
        np.testing.assert_allclose(o["loss"].cpu().numpy(), ref["loss"].cpu().numpy(), rtol=1e-5)
        d, r = o["dw"].cpu().numpy(), ref["dw"].cpu().numpy()
        assert np.linalg.norm(d - r) <= 1e-4 * np.linalg.norm(r), impl
    # the plain clip cascade and the plain unit-gain GMP cascade share the DPD kernels
    assert torch.equal(out["plain"]["u"], ref["u"])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_training_through_clip_pa(prec):
    """Direct learning through the clipping PA lowers the loss."""
    announce(f"training through the clipping PA, prec={prec}")
    inp = S.make_workload("parity_16k")
    wl = inp.workload
    cas = D.ClipCascade(wl.taps, wl.n_hidden, wl.hidden, inp.offsets, 1.2, precision=prec, gain=0.9)
    x = H.to_dev(inp.x)
    w = H.to_dev(inp.w).clone()
    losses = cas.train(x, w, 60)
    torch.cuda.synchronize()
    first, last = float(losses[0, 0]), float(losses[-1, 0])
    print(f"  loss {first:.4e} -> {last:.4e}", flush=True)
    assert last < 0.7 * first
