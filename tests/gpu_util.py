"""Helpers for the GPU parity tests: allocation, calls through the C ABI
binding, host copies and comparisons against the oracle."""
from __future__ import annotations

import sys

import numpy as np
import torch

from paper_1004_3105_amd import binding as nb
from helpers import fp32_tol, fp64_poly_tol, fp64_scaled_tol, half_tol, ulp_dist64_fast

TDT = {nb.NRNG_F64: torch.float64, nb.NRNG_F32: torch.float32, nb.NRNG_BF16: torch.bfloat16,
       nb.NRNG_F16: torch.float16}
NAME = {nb.NRNG_F64: "f64", nb.NRNG_F32: "f32", nb.NRNG_BF16: "bf16", nb.NRNG_F16: "f16"}


def case(*parts) -> None:
    """Name the GPU step about to run (flushed, so it survives a crash)."""
    print("[gpu case]", *parts, flush=True)
    sys.stdout.flush()


def dev():
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


def run(method: str, seed: int, offset: int, n: int, dtype: int, mu: float = 0.0, sigma: float = 1.0,
        out=None, with_consumed: bool = False):
    d = dev()
    if out is None:
        out = torch.empty(max(n, 1), dtype=TDT[dtype], device=d)[:n]
    cons = torch.zeros(1, dtype=torch.int64, device=d)
    case(method, NAME[dtype], "seed", seed, "offset", offset, "n", n, "mu", mu, "sigma", sigma)
    if method == "b1":
        nb.nrng_boxmuller(seed, offset, n, mu, sigma, out, dtype)
    elif method == "b3":
        nb.nrng_b3(seed, offset, n, mu, sigma, out, dtype)
    elif method == "b2":
        nb.nrng_b2(seed, offset, n, mu, sigma, out, dtype)
    elif method == "polar2":
        nb.nrng_polar2(seed, offset, n, mu, sigma, out, dtype, None, cons)
    elif method == "ratio":
        nb.nrng_ratio(seed, offset, n, mu, sigma, out, dtype, None, cons)
    else:
        nb.nrng_polar(seed, offset, n, mu, sigma, out, dtype, None, cons)
    torch.cuda.synchronize()
    if with_consumed:
        return out, int(cons.cpu().numpy().view(np.uint64)[0])
    return out


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().to(torch.float64).cpu().numpy()


def u64(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def assert_close(z: np.ndarray, ref: np.ndarray, dtype: int, mu=0.0, sigma=1.0, what: str = "",
                 poly: bool = False, extra=None):
    """Compare GPU values with the oracle's at the bar of the dtype (poly: the
    FP64 bar of the methods with the Section 3 polynomial, P2 and B3; see
    helpers.fp64_poly_tol; extra: an absolute term added to the FP32 and
    BF16/FP16 bars, per value, as for method B2 in single precision).
    Returns the largest ulp distance (FP64) or the largest fraction of the
    bar (other dtypes)."""
    assert z.shape == ref.shape, (z.shape, ref.shape)
    if dtype == nb.NRNG_F64:
        d = ulp_dist64_fast(z, ref)
        ok = d <= 4
        if poly:
            ok |= np.abs(z - ref) <= fp64_poly_tol(ref, mu, sigma)
        if np.any(mu != 0.0):
            # z = sigma n + mu: four units in the last place of the larger of
            # |z|, |mu| and sigma |n| (for mu = 0 this is the plain 4-ulp bar)
            ok |= np.abs(z - ref) <= fp64_scaled_tol(ref, mu, sigma)
        bad = np.flatnonzero(~ok)
        assert bad.size == 0, "%s: %d values beyond 4 ulp, first at %d: gpu %r ref %r (%d ulp)" % (
            what, bad.size, bad[0], z[bad[0]], ref[bad[0]], d[bad[0]])
        return int(d.max()) if d.size else 0
    if dtype == nb.NRNG_F32:
        tol = fp32_tol(ref, mu, sigma)
    else:
        tol = half_tol(ref, "bf16" if dtype == nb.NRNG_BF16 else "f16", mu, sigma)
    if extra is not None:
        tol = tol + extra
    err = np.abs(z - ref)
    bad = np.flatnonzero(err > tol)
    assert bad.size == 0, "%s: %d values out of tolerance, first at %d: gpu %r ref %r (err %g tol %g)" % (
        what, bad.size, bad[0], z[bad[0]], ref[bad[0]], err[bad[0]], tol[bad[0]])
    return float((err / tol).max()) if err.size else 0.0
