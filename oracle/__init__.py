"""Plain FP64 CPU oracle for the TDNN-DPD -> GMP-PA cascade (arXiv 2205.05158).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import it; the product path never does.  It shares no code
with the HIP library.

parity pins: every function here is checked by tests/test_oracle_pins.py,
tests/test_oracle_grad.py, tests/test_oracle_adam.py (the training loop of
oracle/adam.py), tests/test_oracle_ila.py (the least-squares GMP DPD of
oracle/ila.py), tests/test_oracle_fdcnn.py (the FD-CNN of oracle/fdcnn.py) and
tests/test_oracle_ofdm.py (the FD-NN wrapper, ZF precoding and downlink of
oracle/ofdm.py), tests/test_oracle_clip.py (the linear-clipping PA of
oracle/clip_pa.py) against values fixed independently of the oracle (closed forms,
library routines, brute force, finite differences).  The whole
cascade at full workload sizes is trusted by composition of those pinned parts.
"""
from .dpd_pa import (Model, CascadeResult, advance, cascade, cascade_at, complex_of, db10,
                      delay, features, gmp_backward, gmp_forward, gmp_terms, nmse_parts,
                      pack_tdnn, tdnn_backward, tdnn_forward, unpack_gmp, unpack_tdnn)
from .clip_pa import cascade_clip, clip_backward, clip_forward
from .spectrum import acpr_db, band_powers, hann_periodic, welch_psd

__all__ = [
    "Model", "CascadeResult", "advance", "cascade", "cascade_at", "complex_of", "db10", "delay",
    "features", "gmp_backward", "gmp_forward", "gmp_terms", "nmse_parts", "pack_tdnn",
    "tdnn_backward", "tdnn_forward", "unpack_gmp", "unpack_tdnn", "acpr_db", "band_powers",
    "hann_periodic", "welch_psd", "cascade_clip", "clip_backward", "clip_forward",
]
