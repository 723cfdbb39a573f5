"""Build the gfx950 shared library ``liblb2p.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "liblb2p.so")
SOURCES = [os.path.join(CSRC, "lb2p_api.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("kernels.hpp", "kernels_fused.hpp", "kernels_closure.hpp", "lattice.hpp")] + [
    os.path.join(ROOT, "include", "lb2p.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds fused only within one expression, as written: every
    # rounding follows from the source, the same in every instantiation
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function",
]


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(OUT):
        newest = max(os.path.getmtime(p) for p in SOURCES + HEADERS)
        if os.path.getmtime(OUT) >= newest:
            return OUT
    cmd = [HIPCC, *FLAGS, *SOURCES, "-o", OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT



def source_sha() -> str:
    """Hash of the kernel and ABI sources (ties recorded counters to code)."""
    import hashlib
    h = hashlib.sha256()
    for p in sorted(SOURCES + HEADERS):
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    print(build(force=True, verbose="-v" in sys.argv))
