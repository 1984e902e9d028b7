"""Build libnrng.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Usage: python -m paper_1004_3105_amd.build   (or build() from Python).
The library is written next to this file; it is what the Python binding,
the tests and the benchmark load.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnrng.so")
SOURCES = ["nrng_kernels.hip", "nrng_probes.hip", "nrng_abi.cpp"]
HEADERS = ["nrng_device.hpp", "nrng_launch.hpp", "nrng_p2_poly.hpp", "nrng_b2_poly.hpp"]
ARCH = os.environ.get("NRNG_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Wno-unused-result",
    "-Wno-pass-failed",
    # no packed-FP32 instructions are generated (see the build notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libnrng.so (always recompiles)."""
    hipcc = os.environ.get("HIPCC", "hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc] + HIPCC_FLAGS + ["-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (r.stderr or "").splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed (%d):\n%s" % (r.returncode, err))
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
