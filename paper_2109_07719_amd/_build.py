"""Build step for the HIP library (libabadj.so, in-tree, gfx950 only)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libabadj.so")
CSRC = os.path.join(HERE, "csrc")
HEADERS = [os.path.join(CSRC, n) for n in ("spatial.h", "aba_lane.h", "dual.h", "abadj_device.h",
                                           "abadj_internal.h")] + [os.path.join(ROOT, "include", "abadj.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC",
    # no packed-FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # device code only: let the compiler fold x*0, x+0, x*1 (structural
    # zeros of canonicalised joints); no reassociation.  The host runtime
    # keeps IEEE semantics (its input validation tests for non-finite numbers)
    "-Xarch_device", "-fno-signed-zeros", "-Xarch_device", "-ffinite-math-only",
]
# Translation units (compiled in parallel) and any options of their own.
UNITS = [
    ("abadj_kernels.hip", []),
    ("abadj_kernels_bwd.hip", []),
    ("abadj_kernels_bwd64.hip", []),
    ("abadj_kernels_chain.hip", []),
    ("abadj_runtime.hip", []),
    ("pgs.hip", []),
    ("contact.hip", []),
]
SOURCES = [os.path.join(CSRC, u) for u, _ in UNITS]


def _filter(text: str) -> str:
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops' is not a recognized feature" not in l)


def build_library(verbose: bool = False) -> str:
    """Compile the translation units in parallel, then link libabadj.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs, procs = [], []
    for unit, extra in UNITS:
        obj = os.path.join(CSRC, os.path.splitext(unit)[0] + ".o")
        objs.append(obj)
        cmd = [hipcc, *HIPCC_FLAGS, *extra, "-c", "-o", obj, os.path.join(CSRC, unit)]
        procs.append((unit, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    errors, out = [], []
    for unit, p in procs:
        text = _filter(p.communicate()[0])
        out.append(text)
        if p.returncode != 0:
            errors.append(f"{unit}:\n{text}")
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    res = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs],
                         capture_output=True, text=True)
    out.append(_filter(res.stdout + res.stderr))
    for obj in objs:
        os.remove(obj)
    if res.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + out[-1])
    if verbose and "".join(out).strip():
        print("\n".join(out))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
