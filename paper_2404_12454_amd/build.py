"""Compile the HIP library in-tree for gfx950: ``python -m paper_2404_12454_amd.build``.

The shared object lands next to this file (``libgbd.so``) so that it travels
with the source tree.  Packed FP32 instructions are disabled for every device
compilation unit (``-packed-fp32-ops``)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgbd.so")
SOURCES = ["gbd_api.hip", "gbd_kernels.hip", "gbd_sep.hip", "gbd_batch.hip", "gbd_mlp.hip", "gbd_point.hip",
           "gbd_trace.hip", "gbd_cut.hip", "gbd_sep64.hip", "gbd_probe.hip"]
ARCH = os.environ.get("GBD_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in ordinary VGPRs: with the accumulation registers the
    # register allocator permutes the loop-carried accumulators of the
    # separable form every iteration (v_accvgpr moves per MFMA)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    """Always recompiles (the build check must exercise the compiler)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["hipcc", *HIPCC_FLAGS, "-I", os.path.join(HERE, "..", "include"), *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msgs = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{msgs}")
    if verbose and msgs.strip():
        print(msgs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
