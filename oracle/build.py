"""Compile the oracle (plain C, gcc, OpenMP) into oracle/libkbc_oracle.so."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "kbc_oracle.c")
    out = os.path.join(HERE, "libkbc_oracle.so")
    tmp = out + ".tmp"
    # -ffp-contract=off: no fused multiply-adds, so every product and sum is
    # rounded exactly as written.
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
