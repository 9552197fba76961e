"""Build libdpdmi.so (all HIP sources, gfx950) in place, next to this file.

    python -m paper_2205_05158_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libdpdmi.so")
PEAKS_LIB = os.path.join(HERE, "libdpdpeaks.so")   # unit-throughput probes for bench.py
OBJDIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC",
    # packed FP32 VALU ops are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    f"-I{INCLUDE}", f"-I{CSRC}",
]
SOURCES = ["abi.hip", "plain.hip", "reduce.hip", "gmp.hip", "tdnn.hip", "spectrum.hip", "adam.hip", "ls.hip", "fdcnn.hip",
           "ofdm.hip"]
PEAKS_SOURCES = ["peaks.hip"]
# The TDNN kernels keep every dW accumulator of the deepest model in registers;
# selecting the VGPR form of the MFMA instructions lets the register allocator use the
# accumulation registers for spilling instead of moving those accumulators to scratch
# memory.
TDNN_FLAGS = ["-mllvm", "-amdgpu-mfma-vgpr-form"]
# Generic TDNN shapes: tdnn_gen.hip compiled once per precision and padded width.
GEN_UNITS = [(f"tdnn_gen_{p}_{hp}", ["-DDPD_GEN_PREC=DPD_" + p.upper(), f"-DDPD_GEN_HP={hp}",
                                      f"-DDPD_GEN_FN=tdnn_gen_{p}_{hp}"])
             for p in ("fp32", "bf16") for hp in (128, 64, 32)]
# (object stem, source, extra flags) of every translation unit of libdpdmi.so
UNITS = ([(os.path.splitext(s)[0], s, TDNN_FLAGS if s == "tdnn.hip" else []) for s in SOURCES]
         + [(stem, "tdnn_gen.hip", TDNN_FLAGS + defs) for stem, defs in GEN_UNITS])
PEAKS_UNITS = [(os.path.splitext(s)[0], s, []) for s in PEAKS_SOURCES]


def _compile(unit) -> str:
    stem, src, extra = unit
    obj = os.path.join(OBJDIR, stem + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {stem} ({src}):\n{r.stderr}")
    return obj


def _link(objs, out: str) -> None:
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    # the slowest units (the generic fp32 shapes) first
    units = [u for u in UNITS if u[1] == "tdnn_gen.hip"] + [u for u in UNITS if u[1] != "tdnn_gen.hip"] + PEAKS_UNITS
    with ThreadPoolExecutor(max_workers=min(len(units), os.cpu_count() or 4)) as ex:
        objs = dict(zip([u[0] for u in units], ex.map(_compile, units)))
    _link([objs[u[0]] for u in UNITS], LIB)
    _link([objs[u[0]] for u in PEAKS_UNITS], PEAKS_LIB)
    if verbose:
        print(f"built {LIB} and {PEAKS_LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
