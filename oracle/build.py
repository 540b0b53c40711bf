"""Build the HWFV1 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, FP64, no contraction and no fast-math, so every floating-point
operation in the oracle is the single IEEE-754 operation written in the C
source.
"""
import os
import subprocess
import sys
from pathlib import Path

HERE = Path(__file__).resolve().parent
SRC = HERE / "hwfv1_oracle.c"
LIB = HERE / "liboracle.so"

CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> Path:
    """Compile the oracle (always) and return the library path."""
    tmp = LIB.with_suffix(".so.tmp")
    cmd = ["gcc", *CFLAGS, str(SRC), "-o", str(tmp), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def ensure_built() -> Path:
    """Build only when no library exists yet."""
    if not LIB.exists():
        build()
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
