"""Builds the FP64 CPU oracle (test infrastructure) into oracle/liblbm_oracle.so.

Plain C, no intrinsics, no floating-point contraction, OpenMP over rows only.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")


def build(verbose: bool = False, src: str = SRC, out: str = LIB) -> str:
    """Compiles src (the oracle's source, or an altered copy of it) into out."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11",
           "-Wall", "-Wextra", "-fPIC", "-shared", src, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
