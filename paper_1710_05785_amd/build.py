"""Build libdaic.so for gfx950 with hipcc (in-tree, no JIT cache)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdaic.so")
SOURCES = ["daic_runtime.hip", "daic_pull.hip", "daic_batch.hip", "daic_sched.hip", "daic_sweep.hip",
           "daic_check.hip", "daic_state.hip", "daic_noalloc.hip", "daic_tile.hip"]

# Packed FP32 instructions are disabled for all device code; FP atomics map
# to the hardware instructions (the target memory is coarse-grained).
HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics", "-Wl,--no-undefined",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA results in ordinary VGPRs: the network kernels apply ReLU and BF16
    # conversion to every output, which would otherwise copy each one out of
    # the accumulation registers first
    "-mllvm", "-amdgpu-mfma-vgpr-form",
]


def sources():
    return [os.path.join(HERE, "csrc", s) for s in SOURCES
            if os.path.exists(os.path.join(HERE, "csrc", s))]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into one shared library; returns its path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I",
           os.path.join(HERE, "csrc"), *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
