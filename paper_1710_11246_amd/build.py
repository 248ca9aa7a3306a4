"""Build the HIP libraries in-tree for gfx950 (hipcc cross-compiles without a GPU):
libslabhash.so (the slab hash) and libslabhash_roofs.so (access-pattern microbenchmarks)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "slabhash.hip")
HEADER = os.path.join(ROOT, "include", "slabhash.h")
LIB = os.path.join(PKG, "libslabhash.so")
ROOFS_SRC = os.path.join(PKG, "csrc", "roofs.hip")
ROOFS_LIB = os.path.join(PKG, "libslabhash_roofs.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # keep the compiler from forming packed fp32 instructions (none are wanted here)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _compile(src: str, lib: str, verbose: bool) -> str:
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building %s" % src)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    """Compile csrc/slabhash.hip into libslabhash.so and csrc/roofs.hip into
    libslabhash_roofs.so next to this file. Always recompiles. Returns the slab-hash library."""
    _compile(ROOFS_SRC, ROOFS_LIB, verbose)
    return _compile(SRC, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
