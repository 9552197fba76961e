"""Launch shapes of the tuned path (dpd_tune_set / dpd_autotune) on the GPU: every
compiled forward tile shape, grid choice and GMP tile against the FP64 oracle, with u
and y bitwise independent of the shape, and the autotuner's pick installed and used."""
import sys

import numpy as np
import pytest
import torch

import dpd_synth as S
import gpu_helpers as H

pytestmark = pytest.mark.gpu

# fwd_waves x fwd_wg_per_cu x bwd_wg_per_cu x gmp_tile: every value of each field
SHAPES = [dict(fwd_waves=8, fwd_wg_per_cu=1, bwd_wg_per_cu=1, gmp_tile=256),
          dict(fwd_waves=12, fwd_wg_per_cu=4, bwd_wg_per_cu=2, gmp_tile=512),
          dict(fwd_waves=12, fwd_wg_per_cu=2, bwd_wg_per_cu=1, gmp_tile=256),
          dict(fwd_waves=8, fwd_wg_per_cu=3, bwd_wg_per_cu=2, gmp_tile=512),
          dict(fwd_waves=16, fwd_wg_per_cu=1, bwd_wg_per_cu=1, gmp_tile=256)]


def announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)
    sys.stdout.flush()


def _tensors(inp):
    return H.to_dev(inp.x), H.to_dev(inp.w), H.to_dev(inp.coef)


def _host(out):
    return {k: (None if v is None else v.cpu().numpy()) for k, v in out.items()}


@pytest.mark.parametrize("workload,prec", [("batched_64s", "fp32"), ("batched_64s", "bf16"),
                                           ("bf16_16m", "bf16")])
def test_every_shape_matches_oracle(workload, prec):
    kw = dict(n_streams=5, max_len=7000) if workload == "batched_64s" else dict(max_len=12000)
    announce(f"launch shapes {workload} {kw} prec={prec}")
    inp = S.make_workload(workload, **kw)
    ref = H.oracle_for(inp)
    cas = H.cascade_for(inp, precision=prec)
    x, w, c = _tensors(inp)
    cas.set_tune(None)
    base = _host(cas.run(x, w, c))
    torch.cuda.synchronize()
    try:
        for shape in SHAPES:
            print(f"  shape {shape}", flush=True)
            cas.set_tune(shape)
            assert cas.tune() == shape
            got = _host(cas.run(x, w, c))
            torch.cuda.synchronize()
            assert np.array_equal(got["u"], base["u"]) and np.array_equal(got["y"], base["y"])
            H.check_cascade(inp, got, ref, prec)
    finally:
        cas.set_tune(None)


def test_autotune_installs_and_uses_a_shape():
    announce("autotune batched_64s 5 streams <= 7000 samples")
    inp = S.make_workload("batched_64s", n_streams=5, max_len=7000)
    ref = H.oracle_for(inp)
    cas = H.cascade_for(inp)
    x, w, c = _tensors(inp)
    try:
        pick = cas.autotune(x, w, c, reps=2)
        print(f"  picked {pick}", flush=True)
        assert cas.tune() == pick
        assert pick["fwd_waves"] in (8, 12, 16) and pick["gmp_tile"] in (256, 512)
        assert 1 <= pick["fwd_wg_per_cu"] <= 4 and 1 <= pick["bwd_wg_per_cu"] <= 2
        got = _host(cas.run(x, w, c))
        torch.cuda.synchronize()
        H.check_cascade(inp, got, ref, "fp32")
    finally:
        cas.set_tune(None)


@pytest.mark.parametrize("lens", [[7000, 63, 1, 4097, 2500], [65, 191, 193, 64]],
                         ids=["ragged5", "tile_edges"])
def test_bf16_gradient_independent_of_forward_tile(lens):
    """bf16: the reverse mode reads the hidden activations the forward stored per 16-sample
    group; with the backward grid fixed, dW (and the loss) are bitwise the same whatever
    forward tile (8, 12 or 16 waves, 128/192/256 samples) wrote them, on ragged streams
    whose lengths straddle the 64-sample reverse-mode tiles and the forward tiles."""
    announce(f"bf16 gradient vs forward tile, streams {lens}")
    inp = S.make_workload("batched_64s", n_streams=len(lens), max_len=max(lens))
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    x_np = np.concatenate([inp.x[inp.offsets[s]:inp.offsets[s] + n] for s, n in enumerate(lens)])
    inp = S.Inputs(inp.workload, x_np, off, inp.w[:len(lens)], inp.coef[:len(lens)])
    ref = H.oracle_for(inp)
    cas = H.cascade_for(inp, precision="bf16")
    x, w, c = _tensors(inp)
    outs = []
    try:
        for fw in (8, 12, 16):
            cas.set_tune(dict(fwd_waves=fw, fwd_wg_per_cu=1, bwd_wg_per_cu=1, gmp_tile=256))
            outs.append(_host(cas.run(x, w, c)))
            torch.cuda.synchronize()
    finally:
        cas.set_tune(None)
    for o in outs[1:]:
        assert np.array_equal(o["dw"], outs[0]["dw"]) and np.array_equal(o["loss"], outs[0]["loss"])
    H.check_cascade(inp, outs[0], ref, "bf16")
