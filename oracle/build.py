"""Compile the C oracle (test infrastructure) into oracle/_build/libdd_oracle.so.

Flags keep every FP64 operation a single IEEE-754 operation in source order:
no contraction into FMA, no fast-math, SSE2 doubles (x86-64 default).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dd_oracle.c")
OUT_DIR = os.path.join(HERE, "_build")


def library_path() -> str:
    return os.path.join(OUT_DIR, "libdd_oracle.so")


def build_oracle(verbose: bool = False, src: str = SRC, out: str = None) -> str:
    """Compile ``src`` (default: the oracle) to ``out`` (default: the oracle's
    library path).  Tests use the two arguments to build planted-mistake
    copies of the oracle in a temporary directory."""
    out = out or library_path()
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-fno-unsafe-math-optimizations",
           "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_oracle(verbose="-v" in sys.argv))
