"""Build libnrng.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Usage: python -m paper_1004_3105_amd.build   (or build() from Python).
Each source is compiled to an object in its own hipcc process (in parallel:
the kernel families are separate translation units), then the objects are
linked into the library next to this file; it is what the Python binding,
the tests and the benchmark load.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnrng.so")
SOURCES = ["nrng_kernels_p.hip", "nrng_kernels_r.hip", "nrng_kernels_p2.hip", "nrng_kernels_b1.hip",
           "nrng_kernels_b3.hip", "nrng_kernels_b2.hip", "nrng_kernels_misc.hip", "nrng_probes.hip",
           "nrng_abi.cpp"]
HEADERS = ["nrng_kernels.hpp", "nrng_device.hpp", "nrng_launch.hpp", "nrng_p2_poly.hpp", "nrng_b2_poly.hpp"]
ARCH = os.environ.get("NRNG_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-result",
    "-Wno-pass-failed",
    # no packed-FP32 instructions are generated (see the build notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
NOISE = "is not a recognized feature for this target"


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stderr or "").splitlines() if NOISE not in l)
    return r.returncode, err


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source (always recompiles) and link libnrng.so."""
    hipcc = os.environ.get("HIPCC", "hipcc")
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1, 16)
    objs = [os.path.join(OBJ, os.path.splitext(s)[0] + ".o") for s in SOURCES]

    def compile_one(i):
        return _run([hipcc] + HIPCC_FLAGS + ["-c", "-o", objs[i], os.path.join(CSRC, SOURCES[i])])

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(compile_one, range(len(SOURCES))))
    for src, (rc, err) in zip(SOURCES, results):
        if rc != 0:
            raise RuntimeError("hipcc failed on %s (%d):\n%s" % (src, rc, err))
        if verbose and err.strip():
            print(err, file=sys.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    rc, err = _run([hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    if rc != 0:
        raise RuntimeError("hipcc link failed (%d):\n%s" % (rc, err))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
