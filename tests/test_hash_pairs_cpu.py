"""Integer identities the kernels rely on (CPU, no GPU): even-odd counter
pairs, and the accept test screened on raw hash words.

SplitMix64's first round maps z to (z ^ (z >> 30)) * C1 mod 2^64.  For an
even z and z + 1 the xor-shift results differ in bit 0 only, so the odd
counter's first product is the even one's plus C1 when bit 30 of z is clear
and minus C1 when it is set.  The kernels form the odd counter's hash that
way (one 64-bit add instead of the first round); these checks pin the
identity, including z at the ends of 2^30 and 2^32 blocks, and that it does
not hold in general for an odd z (which the kernels never pair with the
counter after it).
"""
import numpy as np

import synth

M64 = (1 << 64) - 1
C1 = 0xBF58476D1CE4E5B9


def round1(z: int) -> int:
    return ((z ^ (z >> 30)) * C1) & M64


def step(z_even: int) -> int:
    return (-C1) & M64 if (z_even >> 30) & 1 else C1


def test_odd_counter_product_from_the_even_one():
    rng = synth.rng(0x9A1)
    zs = [int(x) & ~1 for x in rng.integers(0, 1 << 63, 20000, dtype=np.uint64)]
    zs += [int(x) << 1 for x in rng.integers(0, 1 << 62, 2000, dtype=np.uint64)]
    edges = []
    for b in (30, 31, 32, 33, 62, 63):
        for k in (1, 2, 3):
            base = (k << b) & M64
            edges += [(base - 2) & M64, base, (base + 2) & M64]
    for z in zs + edges + [0, M64 - 1]:
        assert round1(z + 1 & M64) == (round1(z) + step(z)) & M64, hex(z)


def test_identity_needs_the_even_counter_first():
    # z odd: z + 1 carries into higher bits, and the relation does not hold
    # in general (the kernels never pair an odd counter with the next one)
    for z in ((1 << 30) - 1, (1 << 32) - 1, 0x123456789ABCDEF1, (3 << 40) - 1):
        assert round1(z + 1) != (round1(z) + step(z)) & M64, hex(z)


def _s32(h: int) -> int:
    return h - (1 << 32) if h >= 1 << 31 else h


def test_accept_screen_on_raw_top_words():
    """The mask kernels decide Algorithm P's (and P2's) test on the top words
    h of the two hashes before their final xor-shift (X = h ^ (h >> 31) moves
    only bit 0), and decide exactly only when S' lies within 2^34 of 2^62.
    Outside that band the screened decision equals the exact one, checked on
    random words and on candidates next to the circle s = 1."""
    rng = synth.rng(0x5C2)
    cases = [tuple(int(v) for v in rng.integers(0, 1 << 32, 2, dtype=np.uint64)) for _ in range(100000)]
    t = rng.uniform(0, 2 * np.pi, 100000)
    r = 2.0**31 * (1 + rng.uniform(-2.0**-26, 2.0**-26, t.size))
    for X, Y in zip(np.clip(np.rint(r * np.cos(t)), -2**31, 2**31 - 1), np.clip(np.rint(r * np.sin(t)), -2**31, 2**31 - 1)):
        hx, hy = int(X) & 0xFFFFFFFF, int(Y) & 0xFFFFFFFF
        cases.append((hx ^ 1 if hx >> 31 else hx, hy ^ 1 if hy >> 31 else hy))
    cases += [(0, 0), (1, 0), (0, 1), (0xFFFFFFFF, 0), (0x80000000, 0), (0x80000001, 0x80000000)]
    banded = 0
    for hx, hy in cases:
        X, Y = _s32(hx ^ (hx >> 31)), _s32(hy ^ (hy >> 31))
        S = X * X + Y * Y
        x, y = _s32(hx), _s32(hy)
        sm1 = (x * x + y * y - 1) & M64
        band = ((sm1 - ((1 << 62) - 1 - (1 << 34))) & M64) < (1 << 35)
        banded += band
        if band:
            assert abs(S - (1 << 62)) <= (1 << 35)
            continue
        assert (sm1 < (1 << 62) - 1) == (0 < S < (1 << 62)), (hx, hy)            # P
        assert (((sm1 + 1) & M64) < (1 << 62)) == (S < (1 << 62)), (hx, hy)      # P2
    assert banded > 1000   # the near-circle cases reach the exact path
