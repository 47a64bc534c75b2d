"""Build libtlsph.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtlsph.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("tlsph_kernels.hip", "tlsph_host.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no implicit multiply-add fusion: the hot loops spell out their fma()
    # calls, so every kernel variant rounds the same arithmetic the same way
    "-ffp-contract=off",
    # packed FP32 instructions stay off in all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)


def source_hash() -> str:
    """Short digest of the device sources: counter summaries taken on other
    sources are recognised as stale."""
    import hashlib
    h = hashlib.sha1()
    for f in ("tlsph_kernels.hip", "tlsph_math.h", "tlsph_internal.h"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]
