"""Build the HIP library ``libfmgsr.so`` for gfx950 in-tree.

One hipcc invocation compiles the kernels and the C ABI into a shared
library next to this file.  Flags: gfx950 only; no FMA contraction (every
stencil rounds exactly as written); packed-FP32 instructions disabled.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfmgsr.so")
SOURCES = [os.path.join(CSRC, "fmgsr.hip"), os.path.join(CSRC, "fmgsr_batched.hip")]
HEADERS = [os.path.join(CSRC, "fmgsr_kernels.hpp"), os.path.join(CSRC, "fmgsr_device.hpp"),
           os.path.join(CSRC, "fmgsr_host.hpp"),
           os.path.join(ROOT, "include", "fmgsr.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", LIB + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
