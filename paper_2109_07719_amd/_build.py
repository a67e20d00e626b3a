"""Build step for the HIP library (libabadj.so, in-tree, gfx950 only)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libabadj.so")
SOURCES = [os.path.join(HERE, "csrc", "abadj_kernels.hip"),
           os.path.join(HERE, "csrc", "abadj_runtime.hip")]
HEADERS = [os.path.join(HERE, "csrc", n) for n in ("spatial.h", "aba_lane.h", "abadj_internal.h")] + \
    [os.path.join(ROOT, "include", "abadj.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC", "-shared",
    # no packed-FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # device code only: let the compiler fold x*0, x+0, x*1 (structural
    # zeros of canonicalised joints); no reassociation.  The host runtime
    # keeps IEEE semantics (its input validation tests for non-finite numbers)
    "-Xarch_device", "-fno-signed-zeros", "-Xarch_device", "-ffinite-math-only",
]


def build_library(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
