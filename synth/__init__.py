"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

This module holds none of the method's arithmetic: it only draws workload
parameters and explicit test inputs from NumPy's PCG64 generator with fixed
seeds.  The normal deviates themselves are always driven by the SplitMix64
counter stream, which the oracle and the HIP library each implement on their
own from its published definition.

Workload recipes (the paper has no dataset; its workload is "many deviates,
long vectors"):

* single stream: ``n`` normals from counter ``offset`` of stream ``seed``;
* batched: ``nstreams`` streams whose lengths are log-uniform on
  [1e2, 1e6], means uniform on (-10, 10), standard deviations uniform on
  (0.1, 5), each with its own 64-bit seed, packed back to back in one output
  buffer;
* explicit hash words / integer pairs for the test hooks, including the
  edge cases of each transform.
"""
from __future__ import annotations

import math

import numpy as np

BATCH_SEED = 0xBA7C4


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def batched_streams(nstreams: int = 4096, seed: int = BATCH_SEED, n_lo: float = 1e2, n_hi: float = 1e6,
                    mu_lim: float = 10.0, sigma_lo: float = 0.1, sigma_hi: float = 5.0) -> dict:
    """Per-stream parameters of the batched workload.

    Lengths are floor(10^U) with U uniform on [log10 n_lo, log10 n_hi], capped
    at n_hi; offsets are 0; the output layout is packed (out_off is the
    exclusive prefix sum of the lengths)."""
    g = rng(seed)
    lo, hi = np.log10(n_lo), np.log10(n_hi)
    n = np.minimum(np.floor(10.0 ** g.uniform(lo, hi, nstreams)), n_hi).astype(np.uint64)
    mu = g.uniform(-mu_lim, mu_lim, nstreams)
    sigma = g.uniform(sigma_lo, sigma_hi, nstreams)
    seeds = g.integers(0, 2**64, nstreams, dtype=np.uint64, endpoint=False)
    offset = np.zeros(nstreams, dtype=np.uint64)
    out_off = np.zeros(nstreams, dtype=np.uint64)
    if nstreams > 1:
        out_off[1:] = np.cumsum(n[:-1], dtype=np.uint64)
    return {"n": n, "mu": mu, "sigma": sigma, "seed": seeds, "offset": offset, "out_off": out_off,
            "total": int(n.sum())}


def random_words(count: int, seed: int = 11) -> np.ndarray:
    return rng(seed).integers(0, 2**64, count, dtype=np.uint64, endpoint=False)


def b1_edge_words(seed: int = 12) -> np.ndarray:
    """Explicit 64-bit hash words for the B1 test hook, as (u-word, v-word)
    pairs: exact hand-value inputs, the smallest and largest u, u just
    around 1/2, angles at every eighth of a turn and just beside them, and
    random pairs with u very close to 0 or 1."""
    g = rng(seed)
    T = 1 << 11          # one unit in the last place of a 53-bit uniform
    H = 1 << 63          # u = 1/2
    top = (1 << 64) - T  # u = 1 - 2^-53
    us = [0, T, 2 * T, 3 * T, H - T, H, H + T, 3 << 62, top, top - T, top - 2 * T]
    vs = [(k << 61) + d for k in range(8) for d in (0, T, (1 << 64) - T)]
    vs = [v % (1 << 64) for v in vs]
    pairs = [(u, v) for u in us for v in vs]
    small = g.integers(0, 1 << 40, 256, dtype=np.uint64)
    big = (np.uint64((1 << 64) - 1) - g.integers(0, 1 << 40, 256, dtype=np.uint64))
    rv = g.integers(0, 2**64, 512, dtype=np.uint64, endpoint=False)
    w = np.array(pairs, dtype=np.uint64).reshape(-1)
    w2 = np.stack([np.concatenate([small, big]), rv], axis=1).reshape(-1)
    return np.concatenate([w, w2]).astype(np.uint64)


def polar_edge_xy(seed: int = 13) -> np.ndarray:
    """Explicit int32 candidate pairs (X, Y) for the Polar test hook: the
    hand-value points, the four points on the circle S = 2^62, the origin,
    points one unit inside and outside the circle along both axes and the
    diagonal, small-s points, and dense windows around the circle."""
    g = rng(seed)
    R = 1 << 31
    pts = [(1 << 30, 0), (1 << 30, 1 << 30), (1, 0), (0, 1), (-R, 0), (0, -R), (0, 0),
           (R - 1, 0), (0, R - 1), (-(R - 1), 0), (-R, -R), (-R, R - 1), (R - 1, R - 1),
           (-1, -1), (1, -1), (3, 4), (-R, 1), (1, -R)]
    # points near the circle along the diagonal: X = Y = floor(2^31 / sqrt 2) + d
    c = int(np.floor(R / np.sqrt(2.0)))
    pts += [(c + d, c + e) for d in range(-2, 3) for e in range(-2, 3)]
    pts += [(-(c + d), c + e) for d in range(-2, 3) for e in range(-2, 3)]
    # tiny s (s < 2^-20 <=> S < 2^42 <=> |X|,|Y| below about 2^21)
    small = g.integers(-(1 << 21), 1 << 21, (512, 2))
    # random points on a thin annulus around the circle
    th = g.uniform(0, 2 * np.pi, 4096)
    rad = R * (1.0 + g.uniform(-1e-6, 1e-6, 4096))
    ring = np.stack([np.round(rad * np.cos(th)), np.round(rad * np.sin(th))], axis=1)
    ring = np.clip(ring, -R, R - 1).astype(np.int64)
    uni = g.integers(-R, R, (8192, 2))
    allp = np.concatenate([np.array(pts, dtype=np.int64), small, ring, uni]).astype(np.int64)
    return allp.astype(np.int32).reshape(-1)


def b3_edge_words(seed: int = 15) -> np.ndarray:
    """Explicit 64-bit hash words for the B3 test hook, three per pair
    (u1, u2, u3 words; u = (w >> 11) 2^-53): the hand-value uniforms,
    m = max(u1, u2) within a few units (of 2^-53) of the split u = m^2 = 8/9
    on both sides, m = 0 and m = 1 - 2^-53, angles at every eighth of a turn,
    and random words."""
    g = rng(seed)

    def w(u):   # a word whose top 53 bits are u 2^53 (u a multiple of 2^-53)
        return np.uint64(int(round(u * 2.0**53)) << 11)

    rows = []
    for u1, u2, u3 in ((0.5, 0.25, 0.5), (0.25, 0.5, 0.5), (0.25, 0.5, 0.75), (0.5, 0.25, 0.0),
                       (0.5, 0.5, 0.625), (0.5, 0.5, 0.875), (0.9375, 0.5, 0.5), (0.5, 0.9453125, 0.5),
                       (0.96875, 0.1, 0.5), (0.0, 0.0, 0.3), (1 - 2.0**-53, 0.3, 0.5)):
        rows.append((w(u1), w(u2), w(u3)))
    split = math.isqrt(int(8 * 2**106 // 9))          # about sqrt(8/9) 2^53
    for d in range(-4, 5):
        mk = split + d
        rows.append((np.uint64(mk << 11), np.uint64(int(g.integers(0, mk)) << 11), w(0.3)))
        rows.append((np.uint64(int(g.integers(0, mk)) << 11), np.uint64(mk << 11), w(0.7)))
    for e in range(16):
        rows.append((w(0.6), w(0.2), w(e / 16)))
    arr = np.array(rows, dtype=np.uint64).reshape(-1)
    rnd = g.integers(0, 2**64, 3 * 8192, dtype=np.uint64, endpoint=False)
    return np.concatenate([arr, rnd])


def b2_edge_words(seed: int = 17) -> np.ndarray:
    """Explicit 64-bit hash words for the B2 test hook, as (u-word, v-word)
    pairs: v at every sixteenth of a turn and one unit (of 2^-53, and of the
    top 32 bits) beside it, v across the quarter-turn boundaries of the FP32
    angle reduction, u = 0, 1/2 and 1 - 2^-53 (the largest radius), and
    random words."""
    g = rng(seed)
    T = 1 << 11                       # one unit of a 53-bit uniform
    H = 1 << 32                       # one unit of the top 32 bits
    top = (1 << 64) - T
    us = [0, 1 << 63, top, top - T, 3 << 62]
    vs = []
    for k in range(16):
        base = k << 60
        vs += [(base + d) % (1 << 64) for d in (0, T, -T, H, -H)]
    for b in (1 << 62, 3 << 62):      # quarter-turn boundaries of v - 1/2
        vs += [(b + d) % (1 << 64) for d in (0, T, -T, H, -H, 2 * H, -2 * H)]
    pairs = [(u, v) for u in us for v in vs]
    rv = g.integers(0, 2**64, 2 * 8192, dtype=np.uint64, endpoint=False)
    return np.concatenate([np.array(pairs, dtype=np.uint64).reshape(-1), rv])


def ratio_edge_words(seed: int = 16) -> np.ndarray:
    """Explicit 64-bit hash words for the Algorithm R test hook, two per
    candidate (u-word, v-word; u = (w >> 11) 2^-53): u = 0 with several v;
    u = 1 - 2^-53 with v = 1/2 + k 2^-53 for |k| <= 9 (there
    x = sqrt(8/e) k and the test accepts exactly |k| <= 7); v = 1/2 and the
    extreme v; points 1, 2 and 1024 units of v from the curve
    x^2 = -4 ln(1 - u) on both sides, for random u, and 2^k units away for
    k = 3, 6, ..., 45 (this spans the whole width of any FP32 screening band
    around the curve); and random words."""
    g = rng(seed)
    H = 1 << 52                      # v = 1/2 in units of 2^-53

    def w(k53):                      # word whose top 53 bits are k53
        return np.uint64(int(k53) << 11)

    rows = []
    for vk in (0, H, H - 1, H + 1, (1 << 53) - 1, 3 * (1 << 51)):
        rows.append((w(0), w(vk)))
    top = (1 << 53) - 1              # u = 1 - 2^-53
    for k in range(-9, 10):
        rows.append((w(top), w(H + k)))
    for k53 in (top - 1, top - 1000, (1 << 53) - (1 << 13), 3 * (1 << 51)):
        rows.append((w(k53), w(H)))
        rows.append((w(k53), w(0)))
    c = math.sqrt(8.0 / math.e)
    for uk in g.integers(0, 1 << 53, 96):
        u = int(uk) * 2.0**-53
        lim = math.sqrt(-4.0 * math.log1p(-u)) * (1.0 - u) / c    # |v - 1/2| on the curve
        if lim >= 0.5:
            continue
        for sgn in (1, -1):
            vb = int(round((0.5 + sgn * lim) * 2.0**53))
            for d in (-1024, -2, -1, 0, 1, 2, 1024) + tuple(sg * (1 << k) for k in range(3, 46, 3) for sg in (1, -1)):
                vk = vb + d
                if 0 <= vk < (1 << 53):
                    rows.append((w(uk), w(vk)))
    arr = np.array(rows, dtype=np.uint64).reshape(-1)
    rnd = g.integers(0, 2**64, 2 * 8192, dtype=np.uint64, endpoint=False)
    return np.concatenate([arr, rnd])


def polar2_edge_xy(seed: int = 14) -> np.ndarray:
    """Explicit int32 candidate pairs for the P2 test hook: the Polar edge
    points (which include the origin, accepted by P2), the origin repeated
    inside a word, points whose S = X^2 + Y^2 lies within a few units of
    the split s = 8/9 on both sides, and random points with s in (8/9, 1)
    and in [0, 8/9]."""
    g = rng(seed)
    R = 1 << 31
    base = polar_edge_xy(seed).reshape(-1, 2).astype(np.int64)
    T = (8 * (1 << 62)) // 9
    pts = [(0, 0)] * 5
    # integer points whose S lies within 300 of 8/9 * 2^62, on both sides
    # (found by a search over y; listed so that no search runs here)
    pts += [(2022265419, 98585171), (1993305295, 354979523), (1979349560, 425971572),
            (2021405624, 114872817), (1877914036, 756779581), (1985012704, 398749327),
            (1950686167, 542309818), (1854306938, 812909737), (1880615526, 750041135),
            (1817986653, 891179550), (2022347770, 96881154), (2016019230, 186930268)]
    for y in list(range(0, 64)) + [int(v) for v in g.integers(0, 1 << 28, 64)]:
        x = math.isqrt(T - y * y)
        for d in (-1, 0, 1, 2):
            pts.append((x + d, y))
            pts.append((-(x + d), -y))
    th = g.uniform(0, 2 * np.pi, 4096)
    rad = R * np.sqrt(g.uniform(8.0 / 9.0, 1.0, 4096))
    high = np.stack([np.floor(rad * np.cos(th)), np.floor(rad * np.sin(th))], axis=1)
    high = np.clip(high, -R, R - 1).astype(np.int64)
    rad = R * np.sqrt(g.uniform(0.0, 8.0 / 9.0, 4096))
    low = np.stack([np.floor(rad * np.cos(th)), np.floor(rad * np.sin(th))], axis=1).astype(np.int64)
    allp = np.concatenate([base, np.array(pts, dtype=np.int64), high, low])
    return allp.astype(np.int32).reshape(-1)


def slice_starts(count: int, length: int, span: int, seed: int = 0x51CE) -> np.ndarray:
    """Sorted, even start indices of sampled slices [s, s + length) inside
    [0, span)."""
    g = rng(seed)
    s = g.integers(0, span - length, count)
    return np.sort(s - (s % 2)).astype(np.int64)
