"""Build libqarray.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2404_04994_amd.build          # compile

Each .hip file is compiled to an object, then linked into one shared
library.  The matrix-core scorer gets two extra code-generation options:
relaxed NaN handling (its min reductions need no NaN quieting; no NaN can
arise there) and the VGPR form of the MFMA instructions (results feed VALU
minima directly, no accumulator-register copies).  The IEEE mode bit is left
on: turning it off for one file stops the device library's work-item
queries from inlining into its kernels.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libqarray.so")
OBJ = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]
PER_FILE = {
    "qa_mfma.hip": ["-fno-honor-nans", "-mllvm", "-amdgpu-mfma-vgpr-form=1"],
    # energies are finite: fmin/fmax without NaN canonicalisation
    "qa_batch.hip": ["-fno-honor-nans"],
    # the first kernel arguments arrive in SGPRs at wave start (no scalar load
    # before the first address): the short softargmin and adjoint kernels
    # here gain about 0.2 us each
    "qa_kernels.hip": ["-mllvm", "-amdgpu-kernarg-preload-count=16"],
}


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *PER_FILE.get(os.path.basename(src), []),
           "-I", os.path.join(ROOT, "include"), "-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libqarray.so (always recompiles)."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(4, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
