"""Pins of the FD-CNN oracle (oracle/fdcnn.py): the convolution against
scipy.signal.correlate2d, the whole forward and its gradient against torch (conv2d with
padding, ReLU, linear; autograd) in float64, central finite differences on a tiny
network, closed forms of an identity-like network, the FLOP counts of eqs. (16)-(17),
and planted mistakes."""
import numpy as np
import pytest
import scipy.signal
import torch

import oracle.fdcnn as F

RNG = np.random.default_rng(31)


def rand_case(B=3, n_d=10, side=4, n_conv=2, kc=3):
    s = (RNG.standard_normal((B, n_d)) + 1j * RNG.standard_normal((B, n_d))) / np.sqrt(2)
    w = RNG.standard_normal(F.param_count(n_d, side, n_conv, kc)) * 0.3
    return s, w


def test_to_planes_is_row_major_and_zero_padded():
    s = np.arange(7) + 1j * (10 + np.arange(7))
    x = F.to_planes(s[None], 3)
    assert x.shape == (1, 2, 3, 3)
    assert x[0, 0, 1, 2] == 5 and x[0, 1, 2, 0] == 16 and x[0, 0, 2, 1] == 0 and x[0, 1, 2, 2] == 0


def test_conv_matches_scipy_correlate2d():
    x = RNG.standard_normal((2, 2, 6, 6))
    Wc = RNG.standard_normal((3, 2, 3, 3))
    bc = RNG.standard_normal(3)
    out = F.conv2d_same(x, Wc, bc)
    for b in range(2):
        for o in range(3):
            ref = bc[o] + sum(scipy.signal.correlate2d(x[b, c], Wc[o, c], mode="same") for c in range(2))
            np.testing.assert_allclose(out[b, o], ref, rtol=1e-13, atol=1e-13)


def _torch_net(s, w, n_d, side, n_conv, kc):
    Wc, bc, Wf, bf = (torch.tensor(a, requires_grad=True) for a in F.unpack(w, n_d, side, n_conv, kc))
    st = torch.tensor(s)
    grid = torch.zeros((st.shape[0], side * side), dtype=torch.complex128)
    grid[:, :n_d] = st
    grid = grid.reshape(-1, side, side)
    x = torch.stack([grid.real, grid.imag], dim=1)
    pre = torch.nn.functional.conv2d(x, Wc, bc, padding=kc // 2)
    h = torch.relu(pre).reshape(x.shape[0], -1)
    y = torch.nn.functional.linear(h, Wf, bf)
    return y, (Wc, bc, Wf, bf)


@pytest.mark.parametrize("shape", [dict(n_d=10, side=4, n_conv=2, kc=3), dict(n_d=20, side=5, n_conv=3, kc=5)])
def test_forward_and_gradient_match_torch(shape):
    s, w = rand_case(**shape)
    out, cache = F.forward(s, w, **shape)
    y, params = _torch_net(s, w, **shape)
    n_d = shape["n_d"]
    np.testing.assert_allclose(out, (y[:, :n_d] + 1j * y[:, n_d:]).detach().numpy(), rtol=1e-12, atol=1e-12)
    target = (RNG.standard_normal(s.shape) + 1j * RNG.standard_normal(s.shape))
    L, g = F.mse_to_target(out, target)
    tt = torch.tensor(np.concatenate([target.real, target.imag], 1))
    Lt = ((y - tt) ** 2).sum() / out.size
    Lt.backward()
    assert abs(L - Lt.item()) < 1e-12 * L
    ref = np.concatenate([p.grad.numpy().reshape(-1) for p in params])
    np.testing.assert_allclose(F.backward(g, cache, **shape), ref, rtol=1e-10, atol=1e-13)


def test_gradient_matches_central_differences():
    shape = dict(n_d=5, side=3, n_conv=2, kc=3)
    s, w = rand_case(B=2, **shape)
    target = s * 0.5
    out, cache = F.forward(s, w, **shape)
    _, g = F.mse_to_target(out, target)
    ana = F.backward(g, cache, **shape)
    num = np.zeros_like(w)
    for i in range(w.size):
        e = 1e-6 * max(1.0, abs(w[i]))
        wp = w.copy(); wp[i] += e
        wm = w.copy(); wm[i] -= e
        num[i] = (F.mse_to_target(F.forward(s, wp, **shape)[0], target)[0] -
                  F.mse_to_target(F.forward(s, wm, **shape)[0], target)[0]) / (2 * e)
    assert np.linalg.norm(ana - num) / np.linalg.norm(num) < 1e-6


def test_identity_network_closed_form():
    """Kernel 0 passes Re through (centre tap 1), kernel 1 passes Im; biases 0; the output
    layer picks subcarrier n of each plane: for inputs with positive Re and Im the network
    is the identity (ReLU inactive), and negative parts are cut to 0."""
    n_d, side, kc = 7, 3, 3
    Wc = np.zeros((2, 2, kc, kc)); Wc[0, 0, 1, 1] = 1.0; Wc[1, 1, 1, 1] = 1.0
    Wf = np.zeros((2 * n_d, 2 * side * side))
    for n in range(n_d):
        Wf[n, n] = 1.0
        Wf[n_d + n, side * side + n] = 1.0
    w = np.concatenate([Wc.reshape(-1), np.zeros(2), Wf.reshape(-1), np.zeros(2 * n_d)])
    s = np.abs(RNG.standard_normal((2, n_d))) + 1j * np.abs(RNG.standard_normal((2, n_d)))
    np.testing.assert_allclose(F.forward(s, w, n_d, side, 2, kc)[0], s, rtol=0, atol=0)
    s2 = -s.real + 1j * s.imag
    np.testing.assert_allclose(F.forward(s2, w, n_d, side, 2, kc)[0], 1j * s.imag, rtol=0, atol=0)


def test_paper_configuration_flops_and_sizes():
    """N_d = 384, side 20, N^Conv = 2, K_C = 3: flattened length 800, 768 outputs;
    eq. (16) 2 N^Conv L_U (2 K_C^2 - 1) side^2 = 27,200, eq. (17) 8 N_d L_U side^2 =
    1,228,800 (with L_U = 1, N^Conv = 2 L_U)."""
    n_d, side, n_conv, kc = 384, 20, 2, 3
    assert F.param_count(n_d, side, n_conv, kc) == 36 + 2 + 768 * 800 + 768
    assert 2 * n_conv * 1 * (2 * kc * kc - 1) * side ** 2 == 27200
    assert 2 * (2 * n_d) * (n_conv * side * side) == 8 * n_d * 1 * side ** 2


@pytest.mark.parametrize("mistake", ["flip_kernel", "no_relu_mask", "im_first"])
def test_planted_mistakes_are_caught(monkeypatch, mistake):
    if mistake == "flip_kernel":
        orig = F.conv2d_same
        monkeypatch.setattr(F, "conv2d_same", lambda x, Wc, bc: orig(x, Wc[:, :, ::-1, ::-1], bc))
    elif mistake == "no_relu_mask":
        orig_b = F.backward

        def bwd(g_out, cache, *a, **kw):
            x, pre, h, Wc, Wf = cache
            return orig_b(g_out, (x, np.abs(pre) + 1.0, h, Wc, Wf), *a, **kw)
        monkeypatch.setattr(F, "backward", bwd)
    else:
        orig_p = F.to_planes
        monkeypatch.setattr(F, "to_planes", lambda s, side: orig_p(s, side)[:, ::-1].copy())
    pins = [test_conv_matches_scipy_correlate2d,
            lambda: test_forward_and_gradient_match_torch(dict(n_d=10, side=4, n_conv=2, kc=3)),
            test_identity_network_closed_form]
    caught = 0
    for p in pins:
        try:
            p()
        except AssertionError:
            caught += 1
    assert caught > 0


def test_identity_start_of_the_receiver_training_is_the_identity():
    """The FD-CNN identity weights of the receiver-side training driver map unit-energy
    256-QAM symbol vectors to themselves exactly (checked with the oracle's forward)."""
    import dpd_synth as S
    from paper_2205_05158_amd.train_downlink import identity_fdcnn
    n_d, side, kc = 384, 20, 3
    w = identity_fdcnn(n_d, side, kc)
    s = S.fdcnn_symbols(6, n_d, 256, seed=2)
    z = s[..., 0].astype(np.float64) + 1j * s[..., 1]
    out, _ = F.forward(z, w, n_d, side, 2, kc)
    np.testing.assert_allclose(out, z, atol=1e-6)
