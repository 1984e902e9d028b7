"""Test helpers: golden-file parsing, ulp distances and the tolerances the
parity tests use.  No arithmetic of the method lives here."""
from __future__ import annotations

import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

_MATH_NS = {k: getattr(math, k) for k in ("sqrt", "log", "log1p", "pi", "sin", "cos", "exp")}


def golden_rows(name: str):
    """Rows of a '|'-separated golden file, comments and blank lines skipped."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([c.strip() for c in line.split("|")])
    return rows


def closed_form(expr: str) -> float:
    return float(eval(expr, {"__builtins__": {}}, dict(_MATH_NS)))


def ordinal64(x: np.ndarray) -> np.ndarray:
    """Map doubles to integers that are ordered like the doubles, with +0 and
    -0 mapped to the same integer."""
    b = np.ascontiguousarray(x, dtype=np.float64).view(np.int64)
    return np.where(b >= 0, b, -(b & np.int64(0x7FFFFFFFFFFFFFFF)))


def ulp_dist64(a, b) -> np.ndarray:
    oa = ordinal64(np.asarray(a, dtype=np.float64)).astype(object)
    ob = ordinal64(np.asarray(b, dtype=np.float64)).astype(object)
    return np.array([abs(int(x) - int(y)) for x, y in zip(oa, ob)], dtype=object)


def ulp_dist64_fast(a, b) -> np.ndarray:
    """Vectorised ulp distance (saturating; for values of equal sign or near
    zero, which is all the parity tests need)."""
    oa = ordinal64(np.asarray(a, dtype=np.float64))
    ob = ordinal64(np.asarray(b, dtype=np.float64))
    d = oa.astype(np.float64) - ob.astype(np.float64)   # exact enough to compare with 4
    small = np.abs(d) < 2.0**40
    exact = np.where(small, np.abs(oa - ob), np.int64(2**62))
    return exact


def fp32_tol(z_ref: np.ndarray, mu, sigma) -> np.ndarray:
    """FP32 tolerance: 2e-6 * max(1, |z|), widened to the scale of the
    deviate sigma*|n| and of |mu| when mu != 0 (for mu = 0, sigma = 1 this is
    exactly 2e-6 * max(1, |z_ref|))."""
    z = np.abs(z_ref)
    mu = np.asarray(mu, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        nref = np.where(sigma > 0, (z_ref - mu) / np.where(sigma > 0, sigma, 1.0), 0.0)
    scale = np.maximum.reduce([np.ones_like(z), z, np.abs(mu) * np.ones_like(z), np.abs(sigma * nref)])
    return 2e-6 * scale


def fp64_scaled_tol(z_ref: np.ndarray, mu, sigma) -> np.ndarray:
    """FP64 bar for z = sigma n + mu: 4 ulp of max(|z|, |mu|, sigma |n|).

    With mu = 0 this is the plain 4-ulp bar on z.  With mu != 0 the sum can
    cancel (|z| much smaller than sigma |n|): the kernel's and the oracle's
    n agree to a few ulp of n, which after the cancellation is many ulp of
    z (9 seen), so 4 ulp of |z| alone cannot be met by any correct FP64
    evaluation.  Scaling by the larger of |mu| and sigma |n| bounds the
    error that the final multiply-add itself can leave."""
    z = np.abs(z_ref)
    mu = np.asarray(mu, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        nref = np.where(sigma > 0, (z_ref - mu) / np.where(sigma > 0, sigma, 1.0), 0.0)
    scale = np.maximum.reduce([z, np.abs(mu) * np.ones_like(z), np.abs(sigma * nref)])
    return 4.0 * np.spacing(scale)


def fp64_poly_tol(z_ref: np.ndarray, mu, sigma) -> np.ndarray:
    """FP64 bar for the methods that evaluate the Section 3 polynomial (P2
    and B3): the 4-ulp bar of fp64_scaled_tol plus 4e-15 sigma |n|.  The
    two sides evaluate the same degree-15 polynomial
    h(v) differently: the oracle sums the Chebyshev series by the three-term
    recurrence (measured error up to 6.7e-16 against 40-digit evaluation),
    the kernel uses Horner's rule on the monomial coefficients (2.2e-16);
    h >= 1, so their relative disagreement stays below about 1e-15, and the
    extra 4e-15 sigma |n| leaves a factor of four."""
    z = np.asarray(z_ref, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    return fp64_scaled_tol(z, mu, sigma) + 4e-15 * np.abs(z - mu)


def b2_f32_extra(ref_pairs: np.ndarray, mu, n: int) -> np.ndarray:
    """Extra absolute FP32 tolerance of method B2: after four angle doublings
    in single precision the sine and cosine carry an absolute error of up to
    about 2^-20 (1 - 2 sin^2 cancels near cos = 0; 8.4 2^-24 measured over
    1.7e7 angles, about 24 2^-24 by a rounding-error bound), so each value may
    be off by that times sigma r, r the pair's radius.  ref_pairs holds the
    oracle's complete pairs (even length); the result is cut to n values."""
    d = (np.asarray(ref_pairs, dtype=np.float64) - mu).reshape(-1, 2)
    sr = np.hypot(d[:, 0], d[:, 1])
    return np.repeat(2.0**-19 * sr, 2)[:n]


def ulp_of(x: np.ndarray, dtype) -> np.ndarray:
    """Spacing of the target format at |x| (normal and subnormal range)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    if dtype == "f16":
        e = np.floor(np.log2(np.maximum(x, 2.0**-14)))
        return 2.0 ** (e - 10)
    if dtype == "bf16":
        e = np.floor(np.log2(np.maximum(x, 2.0**-126)))
        return 2.0 ** (e - 7)
    raise ValueError(dtype)


def half_tol(z_ref: np.ndarray, dtype, mu=0.0, sigma=1.0) -> np.ndarray:
    """BF16/FP16 tolerance: one unit in the last place of the target format
    at z_ref plus the FP32 tolerance (the value is computed in FP32 and then
    rounded once to the narrow format)."""
    return ulp_of(z_ref, dtype) + fp32_tol(z_ref, mu, sigma)


def bf16_to_f64(bits: np.ndarray) -> np.ndarray:
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def stat_bounds(N: int) -> dict:
    """Acceptance thresholds for moment and KS checks on N independent
    samples (five standard errors; KS at about the 0.1% level)."""
    return {
        "mean": 5.0 / math.sqrt(N),
        "var": 5.0 * math.sqrt(2.0 / N),
        "skew": 5.0 * math.sqrt(6.0 / N),
        "kurt": 5.0 * math.sqrt(24.0 / N),
        "ks": 1.95 / math.sqrt(N),
    }
