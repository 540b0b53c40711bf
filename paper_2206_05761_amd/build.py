"""Build the HWFV1 HIP library (gfx950) into paper_2206_05761_amd/libhwfv1.so.

Every HIP source is compiled without floating-point contraction (the FP64
path must perform exactly the operations written), with packed FP32
instructions disabled, for gfx950 only.
"""
import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
SRC = [PKG / "csrc" / "hw_kernels.hip", PKG / "csrc" / "hw_api.hip"]
LIB = PKG / "libhwfv1.so"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-mcode-object-version=5",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{ROOT / 'include'}", f"-I{PKG / 'csrc'}",
]


def build(verbose: bool = False) -> Path:
    """Compile the library (always) and return its path."""
    tmp = LIB.with_name(LIB.name + ".tmp")
    cmd = [HIPCC, *FLAGS, *map(str, SRC), "-o", str(tmp)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
