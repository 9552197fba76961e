"""Receiver-side training of the frequency-domain DPDs on one GPU (the supervised setting of
Sec. V-A-2: MSE between the equalised received symbols and the transmitted symbols,
through every simulated block — FD DPD, ZF precoding, per-antenna PAs, channel — Adam
with learning rate 0.001, a new channel realisation for every mini-batch).

Every step runs on the device (forward chain, reverse mode of link and precoding, the
network's reverse mode, Adam).  Inputs are seeded synthetic (dpd_synth); no receiver
noise, so the error left is the PA distortion and the CSI error.  Prints one JSON line
per evaluation (receiver MSE and symbol error rate on held-out OFDM symbols and
channels, for the trained network and for no DPD) and a summary line with the time per
step.

    python -m paper_2205_05158_amd.train_downlink --net fdcnn --steps 2000 --eval-every 500
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time


def identity_fdcnn(n_d: int, side: int, kc: int, beta: float = 2.0):
    """FD-CNN weights (two kernels) that map the symbols to themselves: kernel 0 takes the
    Re plane's centre tap, kernel 1 the Im plane's, both with bias beta, so ReLU(x + beta)
    = x + beta for |x| < beta (unit-energy QAM stays inside); the output layer picks
    plane 0 / plane 1 at the symbol's grid position and subtracts beta."""
    import numpy as np
    F = 2 * side * side
    wc = np.zeros((2, 2, kc, kc))
    wc[0, 0, kc // 2, kc // 2] = 1.0
    wc[1, 1, kc // 2, kc // 2] = 1.0
    wf = np.zeros((2 * n_d, F))
    for n in range(n_d):
        wf[n, n] = 1.0
        wf[n_d + n, side * side + n] = 1.0
    return np.concatenate([wc.reshape(-1), [beta, beta], wf.reshape(-1),
                           np.full(2 * n_d, -beta)]).astype(np.float32)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--net", default="fdcnn", choices=["fdcnn", "fdnn"])
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--eval-every", type=int, default=250)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=10, help="OFDM symbols per mini-batch")
    ap.add_argument("--eval-sym", type=int, default=64)
    ap.add_argument("--n-fft", type=int, default=4096)
    ap.add_argument("--n-data", type=int, default=384)
    ap.add_argument("--users", type=int, default=8)
    ap.add_argument("--antennas", type=int, default=32)
    ap.add_argument("--taps", type=int, default=10)
    ap.add_argument("--qam", type=int, default=256)
    ap.add_argument("--eta", type=float, default=1e-4)
    ap.add_argument("--rms", type=float, default=0.3, help="per-antenna time-domain rms at the PA input")
    ap.add_argument("--pa-scale", type=float, default=0.1, help="scale of the synthetic PA's memory/nonlinear terms")
    ap.add_argument("--init", default="xavier", choices=["xavier", "identity"],
                    help="FD-CNN start: Glorot, or the identity map (see identity_fdcnn)")
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    import dpd_synth as S
    from . import _lib as L
    from .downlink import Downlink, FdNn, receiver_loss_grad, receiver_loss_grad_fdcnn
    from .fdcnn import FdCnn

    if not torch.cuda.is_available():
        raise SystemExit("training runs on the GPU")
    N, n_d, U, B, T = args.n_fft, args.n_data, args.users, args.antennas, args.taps
    pa_orders = (7, 3, 1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dl = Downlink(N, n_d, U, B, T, args.qam, pa=pa_orders)
    pa = dev(S.antenna_pa_coefficients(B, *pa_orders, 10, scale=args.pa_scale))
    p_total = args.rms ** 2 * B * N / n_d
    nmax = max(args.batch, args.eval_sym)
    if args.net == "fdnn":
        net = FdNn(N, U, 3, 15, 1, max_sym=nmax)
        w = dev(S.xavier_fdnn(U, 3, 15, 1, 1))
        crit, all_bins = receiver_loss_grad, True
    else:
        side = math.ceil(math.sqrt(n_d))
        net = FdCnn(n_d, side, 2, 3, max_items=nmax * U)
        w0 = identity_fdcnn(n_d, side, 3) if args.init == "identity" else S.xavier_fdcnn(n_d, side, 2, 3, 1)
        w = dev(w0)
        crit, all_bins = receiver_loss_grad_fdcnn, False
    m, v = torch.zeros_like(w), torch.zeros_like(w)

    # held-out evaluation set: its own symbols, channels and noise
    e_idx, e_s = S.downlink_symbols(args.eval_sym, U, N, n_d, args.qam, 7_000)
    e_h, e_he = S.mimo_channel(args.eval_sym, T, U, B, args.eta, 7_001)
    e_s, e_h, e_he, e_tx = dev(e_s), dev(e_h), dev(e_he), torch.from_numpy(e_idx).cuda()
    e_pt, e_alpha = dl.zf(e_he, p_total, all_bins=all_bins)
    bins = torch.as_tensor([*range(1, n_d // 2 + 1), *range(N - n_d // 2, N)], device="cuda")
    n_eval = args.eval_sym * U * n_d

    def evaluate(with_dpd):
        if with_dpd:
            loss, _, err = crit(dl, net, e_s, e_tx, w, e_pt, e_alpha, pa, 1.0, e_h, 1)
            return float(loss), int(err.sum()) / n_eval
        x = dl.precode(e_s, e_pt, e_alpha, all_bins=False)
        err, r = dl.link(x, pa, 1.0, e_h, e_alpha, e_tx, want_r=True)
        d = r - e_s.index_select(2, bins)
        return float((d * d).sum() / n_eval), int(err.sum()) / n_eval

    base_mse, base_ser = evaluate(False)
    print(json.dumps({"net": "none", "receiver_mse": base_mse, "receiver_mse_db": 10 * math.log10(base_mse),
                      "ser": base_ser}), flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_train = 0.0
    for step in range(args.steps + 1):
        if step % args.eval_every == 0 or step == args.steps:
            torch.cuda.synchronize()
            t_train += time.perf_counter() - t0
            mse, ser = evaluate(True)
            print(json.dumps({"net": args.net, "step": step, "receiver_mse": mse,
                              "receiver_mse_db": 10 * math.log10(mse), "ser": ser}), flush=True)
            t0 = time.perf_counter()
        if step == args.steps:
            break
        # a new mini-batch of symbols and a new channel realisation per step
        idx, s = S.downlink_symbols(args.batch, U, N, n_d, args.qam, 10_000 + step)
        h, he = S.mimo_channel(args.batch, T, U, B, args.eta, 20_000 + step)
        s, h, he, tx = dev(s), dev(h), dev(he), torch.from_numpy(idx).cuda()
        pt, alpha = dl.zf(he, p_total, all_bins=all_bins)
        _, dw, _ = crit(dl, net, s, tx, w, pt, alpha, pa, 1.0, h, 1)
        L.dpd_adam_step(dw, w, m, v, step + 1, lr=args.lr)
    torch.cuda.synchronize()
    t_train += time.perf_counter() - t0
    print(json.dumps({"summary": True, "net": args.net, "steps": args.steps, "batch_symbols": args.batch,
                      "ms_per_step_incl_host_inputs": 1e3 * t_train / max(args.steps, 1),
                      "no_dpd_mse_db": 10 * math.log10(base_mse), "no_dpd_ser": base_ser}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
