"""Build the HIP library (gfx950) in-tree with hipcc.

The shared library ``libraytheia_hip.so`` lands next to this file; the
Python binding loads it from there.  Every call recompiles.
"""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_NAME = "libraytheia_hip.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
ARCH = "gfx950"

SOURCES = ["rt_walk.hip", "rt_fields.hip", "rt_accuracy.hip", "rt_build.hip", "rt_octree_dev.hip",
           "rt_calib.hip", "rt_abi.cpp", "rt_octree.cpp"]

# -ffp-contract=off: the walk's FP64 arithmetic must round exactly as written
# (fused multiply-adds only where fma() is spelled out).
# -packed-fp32-ops off: no packed FP32 instructions are generated.
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-I", INCLUDE,
    "-I", CSRC,
]


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return path


def build(verbose=False, extra_flags=()):
    """Compile the library; returns its path."""
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc(), *FLAGS, *extra_flags, *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed with status {r.returncode}")
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
