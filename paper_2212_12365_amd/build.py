"""Builds the HIP library liblesmi.so for gfx950 in-tree with hipcc.

Packed FP32 instructions are disabled for every HIP translation unit
(-target-feature -packed-fp32-ops)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblesmi.so")
SOURCES = ["lesmi.hip", "les_stage.hip", "les_batch.hip", "les_mlp.hip", "les_fwh.hip"]
HEADERS = ["les_device.h", "les_common.h", "les_stage.h", "les_bcdt.h", "les_mlp.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# -amdgpu-mfma-vgpr-form: MFMA results go to ordinary VGPRs rather than AGPRs, which saves
# the accumulator-to-VGPR moves in the closure's inference kernel (the only MFMA code).
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-ffp-contract=off", "-Wl,-z,defs",
         "-mllvm", "-amdgpu-mfma-vgpr-form=1"]


def build(verbose=False):
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
