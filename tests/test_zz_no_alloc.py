"""The allocation-free NMSE entry point (cascade_nmse_noalloc, for callers that cannot
allocate device memory) against cascade_nmse with a caller workspace: the same records,
bit for bit, on two calls in a row, the second with a smaller problem (the static scratch
keeps the first call's partials)."""
import sys

import numpy as np
import pytest
import torch

import dpd_synth as S
import gpu_helpers as H
import paper_2205_05158_amd as D
from paper_2205_05158_amd import _lib as L

pytestmark = pytest.mark.gpu


def _records_both_ways(inp):
    cas = H.cascade_for(inp)
    x = H.to_dev(inp.x)
    y = cas.run(x, H.to_dev(inp.w), H.to_dev(inp.coef), want_grad=False)["y"]
    ref = cas.nmse(y, x)
    out = torch.full((cas.S + 1, D.DPD_NMSE_FIELDS), float("nan"), dtype=torch.float32, device="cuda")
    L.cascade_nmse_noalloc(cas.batch, y, x, cas.gain, out)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_nmse_matches_workspace_call_twice():
    print("\n[gpu case] cascade_nmse_noalloc: 6 streams, then 1 shorter stream", flush=True)
    sys.stdout.flush()
    big = S.make_workload("batched_64s", n_streams=6, max_len=50000)
    small = S.make_workload("parity_16k", max_len=3001)
    got1, ref1 = _records_both_ways(big)
    np.testing.assert_array_equal(got1, ref1)
    got2, ref2 = _records_both_ways(small)
    np.testing.assert_array_equal(got2, ref2)
    assert got2.shape == (2, D.DPD_NMSE_FIELDS) and np.all(np.isfinite(got2[:, :3]))
