"""The identity behind the kernels' even-odd counter pairs (CPU, no GPU).

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
