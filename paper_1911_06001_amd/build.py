"""Build libsvo.so (HIP, gfx950) in place with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsvo.so")
SOURCES = [os.path.join(HERE, "csrc", "svo_host.cpp"), os.path.join(HERE, "csrc", "svo_trace.hip"),
           os.path.join(HERE, "csrc", "svo_raygen.hip")]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         # keep hipcc from emitting packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # every atomic in the kernels is issued by one lane or to per-lane
         # addresses: the pass that merges a wave's atomics only adds code
         "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
         "-Wall", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]


CEILING_LIB = os.path.join(HERE, "libsvo_ceiling.so")
CEILING_SOURCES = [os.path.join(HERE, "csrc", "svo_ceiling.hip")]


def _hipcc(sources, out: str, verbose: bool):
    tmp = out + ".tmp"
    cmd = ["hipcc"] + FLAGS + sources + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    if verbose and errs:
        print("\n".join(errs))
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compile libsvo.so (the trace library) and libsvo_ceiling.so (memory
    ceilings for its roofline)."""
    _hipcc(SOURCES, LIB, verbose)
    _hipcc(CEILING_SOURCES, CEILING_LIB, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
