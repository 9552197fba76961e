"""TD-GMP DPD by indirect learning with least squares on the device (gmp_ls_fit) against
the FP64 oracle of oracle/ila.py: the normal equations entry by entry, the solved
coefficients, whole ILA runs, per-stream sets with ragged lengths, the rank-deficient
case and a linear PA's closed-form post-inverse."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import oracle.ila as OI
import dpd_synth as S
import paper_2205_05158_amd as D
import gpu_helpers as H

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)
    sys.stdout.flush()


def _check_normal(got, ref_G, ref_b):
    """Entries within 1e-11 of the diagonal scale sqrt(G_ii G_jj) (float64 sums of ~1e4
    terms in two different orders)."""
    Gg = got[..., 0] + 1j * got[..., 1]
    d = np.sqrt(np.abs(np.diag(ref_G)).real)      # column norms (0 for an all-zero column)
    assert np.all(np.abs(Gg[:, :-1] - ref_G) <= 1e-11 * np.outer(d, d))
    tn = np.sqrt(np.abs(ref_b).max())              # scale of the target column
    assert np.all(np.abs(Gg[:, -1] - ref_b) <= 1e-9 * d * max(tn, 1.0))


# The raw GMP basis is badly conditioned (cond(Phi^H Phi) ~ 5e9 for (5, 3, 2), 5e12 for
# (7, 5, 3), 6e16 for (9, 7, 4) on this input), so the solution is compared where a ridge
# bounds the condition number by about J / ridge; the normal equations themselves are
# compared entry by entry in every case.
@pytest.mark.parametrize("orders,ridge", [((5, 3, 2), 0.0), ((7, 5, 3), 1e-7), ((9, 7, 4), 1e-7),
                                          ((4, 0, 0), 0.0), ((3, 2, 0), 0.0), ((2, 0, 3), 0.0)])
def test_normal_equations_and_solution_match_oracle(orders, ridge):
    announce(f"ls fit orders={orders} ridge={ridge}")
    inp = S.make_workload("fwd_4m", max_len=20000)
    K, M, Lg = orders
    pa = S.gmp_coefficients(K, M, Lg, seed=5).astype(np.float64)
    # PA input at half the unit RMS (peaks ~1.5) keeps |z|^(K-1) and the conditioning
    # of the normal equations moderate
    t = (0.5 * inp.x).astype(np.float32)       # post-inverse target: the PA input
    y = S.to_interleaved(OI.gmp_apply(t, inp.offsets, pa, K, M, Lg)).astype(np.float32)
    g = complex(np.float32(0.95), np.float32(0.05))   # the float32 gain the library receives
    (ref_c, ref_G, ref_b), = OI.ls_fit(y, t, inp.offsets, K, M, Lg, G=g, ridge=ridge)
    ila = D.GmpIla(orders, orders, inp.offsets, gain=g)
    coef, info, normal = ila.fit(H.to_dev(y), H.to_dev(t), ridge, want_normal=True)
    torch.cuda.synchronize()
    assert int(info.cpu()[0]) == 0
    _check_normal(normal.cpu().numpy()[0], ref_G, ref_b)
    c = coef.cpu().numpy()[0].astype(np.float64)
    rel = np.linalg.norm(c - ref_c) / np.linalg.norm(ref_c)
    cond = np.linalg.cond(ref_G + ridge * np.trace(ref_G).real / ref_G.shape[0] * np.eye(ref_G.shape[0]))
    print(f"  coefficient rel err {rel:.2e} (cond {cond:.1e})", flush=True)
    # float64 solve: cond * 2^-52 (x a modest factor), then rounded to float32
    assert rel <= 1e-6 + 64 * cond * 2.0 ** -52


def test_ila_run_matches_oracle():
    announce("ILA 3 iterations, GMP (5, 3, 2) PA and DPD, 16384 samples")
    inp = S.make_workload("fwd_4m", max_len=16384)
    orders = (5, 3, 2)
    pa = S.gmp_coefficients(*orders, seed=9).astype(np.float64)
    ref_hist, ref_dpd = OI.ila(inp.x, inp.offsets, pa, orders, orders, 3)
    ila = D.GmpIla(orders, orders, inp.offsets)
    hist, dpd, info = ila.run(H.to_dev(inp.x), H.to_dev(pa.astype(np.float32)), 3)
    torch.cuda.synchronize()
    h = hist.cpu().numpy()
    print(f"  NMSE dB gpu {np.round(h, 3)} oracle {np.round(ref_hist, 3)}", flush=True)
    assert int(info.cpu()[0]) == 0
    assert np.max(np.abs(h - ref_hist)) <= H.FP32_NMSE_DB
    assert h[-1] < h[0] - 3.0


def test_per_stream_sets_ragged_and_rank_deficient():
    """Three streams with their own post-distorters, one of 2 samples: its basis columns
    of memory l = 2 are exactly zero, so with ridge 0 its factorisation reports the
    failing pivot and zero coefficients; with a ridge every set matches the oracle."""
    announce("ls fit per-stream sets, lengths 3000 / 2 / 1777")
    lens = [3000, 2, 1777]
    orders = (4, 2, 1)
    K, M, Lg = orders
    rng = np.random.default_rng(12)
    xs = [S.ofdm_signal(4096, 1024, 1, 64, np.random.default_rng(50 + i))[:n] for i, n in enumerate(lens)]
    x = S.to_interleaved(np.concatenate(xs)).astype(np.float32)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    pas = np.stack([S.gmp_coefficients(K, M, Lg, seed=60 + i) for i in range(3)]).astype(np.float64)
    y = S.to_interleaved(OI.gmp_apply(x, off, pas, K, M, Lg, per_stream=True)).astype(np.float32)
    ila = D.GmpIla(orders, orders, off, per_stream_params=True)
    coef, info, _ = ila.fit(H.to_dev(y), H.to_dev(x), 0.0)
    torch.cuda.synchronize()
    inf = info.cpu().numpy()
    assert inf[0] == 0 and inf[2] == 0 and inf[1] > 0
    assert np.all(coef.cpu().numpy()[1] == 0)
    ridge = 1e-6
    refs = OI.ls_fit(y, x, off, K, M, Lg, per_stream=True, ridge=ridge)
    coef, info, normal = ila.fit(H.to_dev(y), H.to_dev(x), ridge, want_normal=True)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    for s, (rc, rG, rb) in enumerate(refs):
        _check_normal(normal.cpu().numpy()[s], rG, rb)
        c = coef.cpu().numpy()[s].astype(np.float64)
        assert np.linalg.norm(c - rc) / np.linalg.norm(rc) <= 1e-5


def test_linear_pa_post_inverse_closed_form():
    """PA y = alpha u from the identity DPD: the fit is a_00 = G / alpha, all else 0."""
    announce("linear PA post-inverse")
    inp = S.make_workload("fwd_4m", max_len=4096)
    orders = (3, 1, 1)
    alpha = 0.7 - 0.2j
    g = complex(np.float32(1.1), np.float32(0.3))
    J = S.gmp_coeff_count(*orders)
    pa = np.zeros((J, 2), np.float32); pa[0] = [alpha.real, alpha.imag]
    ila = D.GmpIla(orders, orders, inp.offsets, gain=g)
    hist, dpd, info = ila.run(H.to_dev(inp.x), H.to_dev(pa), 1)
    torch.cuda.synchronize()
    c = dpd.cpu().numpy()[0]
    want = g / alpha
    np.testing.assert_allclose(c[0], [want.real, want.imag], rtol=2e-6)
    assert np.abs(c[1:]).max() < 1e-6
    assert float(hist.cpu()[-1]) < -100.0


def test_full_size_ila_4m_normal_equations():
    """The bench workload (2^22 samples, GMP (7, 5, 3) DPD and PA, identity DPD): the
    device normal equations against the oracle's, accumulated over chunks of the whole
    stream (bounded memory)."""
    announce("ila_4m full size: normal equations of the first ILA iteration")
    inp = S.make_workload("fwd_4m")
    orders = (7, 5, 3)
    u = inp.x                                           # identity DPD
    y = S.to_interleaved(OI.gmp_apply(u, inp.offsets, inp.coef, *orders)).astype(np.float32)
    print("  oracle PA output ready", flush=True)
    ila = D.GmpIla(orders, orders, inp.offsets)
    coef, info, normal = ila.fit(H.to_dev(y), H.to_dev(u), 0.0, want_normal=True)
    torch.cuda.synchronize()
    assert int(info.cpu()[0]) == 0
    yc = y[:, 0].astype(np.float64) + 1j * y[:, 1]
    uc = u[:, 0].astype(np.float64) + 1j * u[:, 1]
    G, b = OI.normal_equations_chunked(yc, uc, *orders, chunk=1 << 16)
    print("  oracle normal equations ready", flush=True)
    _check_normal(normal.cpu().numpy()[0], G, b)
