"""FD-CNN DPD on the device (fdcnn_forward / fdcnn_backward) against the FP64 oracle of
oracle/fdcnn.py: the paper's configuration (384 data subcarriers on a 20 x 20 grid, two
3 x 3 kernels, ReLU, 800 -> 768 output layer) and another shape, batches that span
several GEMM tiles with a ragged tail, and a short Adam training run."""
import sys

import numpy as np
import pytest
import torch

import oracle.adam as OA
import oracle.fdcnn as OF
import dpd_synth as S
import paper_2205_05158_amd as D
import gpu_helpers as H

pytestmark = pytest.mark.gpu

SHAPES = [dict(n_d=384, side=20, n_conv=2, kc=3), dict(n_d=20, side=5, n_conv=3, kc=5)]


def announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)
    sys.stdout.flush()


def _cplx(a):
    a = np.asarray(a, dtype=np.float64)
    return a[..., 0] + 1j * a[..., 1]


def _rel_l2(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("shape,items", [(SHAPES[0], 70), (SHAPES[0], 1), (SHAPES[1], 130),
                                         (dict(n_d=30, side=6, n_conv=4, kc=1), 65),
                                         (dict(n_d=9, side=3, n_conv=1, kc=7), 33)])
def test_forward_and_backward_match_oracle(shape, items):
    """float32 (matrix cores for the output layer, K = 800) against float64: outputs per
    symbol within 1e-5 of max(|ref|, rms(ref)); each parameter tensor's gradient within
    1e-4 in relative L2 (the FP32 bounds of the TDNN path)."""
    announce(f"fdcnn {shape} items={items}")
    s = S.fdcnn_symbols(items, shape["n_d"], 256, seed=items)
    w = S.xavier_fdcnn(**shape, seed=3)
    rng = np.random.default_rng(items + 1)
    w[shape["n_conv"] * 2 * shape["kc"] ** 2:shape["n_conv"] * (2 * shape["kc"] ** 2 + 1)] = \
        0.1 * rng.standard_normal(shape["n_conv"])            # non-zero conv biases
    g = (rng.standard_normal(s.shape) / items).astype(np.float32)
    ref_out, cache = OF.forward(_cplx(s), w, **shape)
    ref_dw = OF.backward(_cplx(g), cache, **shape)
    net = D.FdCnn(**shape, max_items=items)
    out = net.forward(H.to_dev(s), H.to_dev(w))
    dw = net.backward(H.to_dev(s), H.to_dev(w), H.to_dev(g))
    torch.cuda.synchronize()
    e = H.per_sample_rel(out.cpu().numpy().reshape(-1, 2), ref_out.reshape(-1))
    nc = shape["n_conv"] * 2 * shape["kc"] ** 2
    F = shape["n_conv"] * shape["side"] ** 2
    cuts = [0, nc, nc + shape["n_conv"], nc + shape["n_conv"] + 2 * shape["n_d"] * F, ref_dw.size]
    got = dw.cpu().numpy().astype(np.float64)
    errs = [_rel_l2(got[a:b], ref_dw[a:b]) for a, b in zip(cuts[:-1], cuts[1:])]
    print(f"  output rel err {e:.2e}; gradient rel err per tensor {np.round(errs, 8)}", flush=True)
    assert e <= H.FP32_SAMPLE
    assert max(errs) <= H.FP32_GRAD


def test_training_run_matches_oracle():
    """Five Adam steps (lr 0.001) towards target symbols: the loss before every step within
    1e-4 relative of the oracle's, the total weight change within 1 % in L2."""
    shape = SHAPES[1]
    items, steps = 40, 5
    announce(f"fdcnn training {shape} items={items} steps={steps}")
    s = S.fdcnn_symbols(items, shape["n_d"], 256, seed=5)
    t = S.fdcnn_symbols(items, shape["n_d"], 256, seed=6)
    w0 = S.xavier_fdcnn(**shape, seed=4)
    wr, m, v = w0.astype(np.float64), np.zeros(w0.size), np.zeros(w0.size)
    ref_losses = []
    for k in range(1, steps + 1):
        out, cache = OF.forward(_cplx(s), wr, **shape)
        Lk, gk = OF.mse_to_target(out, _cplx(t))
        ref_losses.append(Lk)
        wr, m, v = OA.adam_step(wr, m, v, OF.backward(gk, cache, **shape), k)
    net = D.FdCnn(**shape, max_items=items)
    w = H.to_dev(w0)
    losses, _ = net.train(H.to_dev(s), w, H.to_dev(t), steps)
    torch.cuda.synchronize()
    got = losses.cpu().numpy()
    print(f"  loss gpu {got} oracle {np.array(ref_losses)}", flush=True)
    np.testing.assert_allclose(got, ref_losses, rtol=1e-4)
    dg = w.cpu().numpy().astype(np.float64) - w0
    dr = wr - w0
    assert _rel_l2(dg, dr) <= 1e-2


def test_autograd_function_with_a_torch_loss():
    """FdCnnFn under a loss written in torch (a fixed complex gain per subcarrier applied
    to the network output, then MSE to target symbols): the gradient torch delivers to w
    equals the oracle's reverse mode for the same output gradient."""
    shape = SHAPES[0]
    items = 24
    announce(f"fdcnn autograd {shape} items={items}")
    s = S.fdcnn_symbols(items, shape["n_d"], 256, seed=7)
    t = S.fdcnn_symbols(items, shape["n_d"], 256, seed=8)
    w0 = S.xavier_fdcnn(**shape, seed=9)
    rng = np.random.default_rng(10)
    hk = (rng.standard_normal(shape["n_d"]) + 1j * rng.standard_normal(shape["n_d"])) / np.sqrt(2)
    net = D.FdCnn(**shape, max_items=items)
    w = H.to_dev(w0).requires_grad_(True)
    out = D.FdCnnFn.apply(w, H.to_dev(s), net)
    oc = torch.complex(out[..., 0].double(), out[..., 1].double())
    hkt = torch.tensor(hk, device="cuda")
    tc = torch.tensor(_cplx(t), device="cuda")
    loss = ((oc * hkt - tc).abs() ** 2).sum() / oc.numel()
    loss.backward()
    torch.cuda.synchronize()
    ref_out, cache = OF.forward(_cplx(s), w0, **shape)
    e = ref_out * hk - _cplx(t)
    g = 2.0 * e * np.conj(hk) / e.size                 # real-convention dL/dout
    ref = OF.backward(g, cache, **shape)
    rel = _rel_l2(w.grad.cpu().numpy().astype(np.float64), ref)
    print(f"  autograd gradient rel err {rel:.2e}", flush=True)
    assert rel <= H.FP32_GRAD


def test_full_size_fdcnn_8u():
    """The bench workload: 8 UEs x 1024 symbol vectors, the paper's network, every output
    and the whole gradient against the oracle."""
    shape = SHAPES[0]
    items = 8 * 1024
    announce(f"fdcnn_8u full size {items} items")
    s = S.fdcnn_symbols(items, shape["n_d"], 256, seed=1)
    w = S.xavier_fdcnn(**shape, seed=2)
    g = (np.random.default_rng(3).standard_normal(s.shape) / items).astype(np.float32)
    ref_out, cache = OF.forward(_cplx(s), w, **shape)
    ref_dw = OF.backward(_cplx(g), cache, **shape)
    net = D.FdCnn(**shape, max_items=items)
    out = net.forward(H.to_dev(s), H.to_dev(w))
    dw = net.backward(H.to_dev(s), H.to_dev(w), H.to_dev(g))
    torch.cuda.synchronize()
    e = H.per_sample_rel(out.cpu().numpy().reshape(-1, 2), ref_out.reshape(-1))
    rel = _rel_l2(dw.cpu().numpy().astype(np.float64), ref_dw)
    print(f"  output rel err {e:.2e}; gradient rel err {rel:.2e}", flush=True)
    assert e <= H.FP32_SAMPLE and rel <= H.FP32_GRAD
