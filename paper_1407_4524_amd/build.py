"""Build step of the HIP library: compiles csrc/*.hip for gfx950 with hipcc
into ``liblbm.so`` next to this file (in-tree, so it travels with the
source tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["kernels.hip", "lbm_api.hip", "batch_api.hip"]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")


def compile_library(verbose: bool = False) -> str:
    out = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           # packed FP32 instructions are kept out of the generated code
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", out] + [os.path.join(HERE, "csrc", s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        sys.stderr.write(msgs + "\n")
        raise RuntimeError("hipcc failed")
    os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    print(compile_library(verbose=True))
