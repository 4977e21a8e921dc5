"""Build the FP64 CPU oracle (test infrastructure only).

Compiles ``fmgsr_oracle.c`` (Poisson) and ``fmgsr_oracle_reaction.c``
(reaction operators, adjoint) with gcc into ``liboracle_fmgsr.so`` next to
them.
Contraction of a*b+c into fused multiply-adds is disabled so that every
stencil rounds exactly as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "fmgsr_oracle.c"), os.path.join(HERE, "fmgsr_oracle_reaction.c")]
LIB = os.path.join(HERE, "liboracle_fmgsr.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", *SRCS, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
