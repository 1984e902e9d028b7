"""Streams placed on the boundaries of the kernels' hashing modes (GPU).

The kernels hash a tile's counters on the low word of z = c + gamma when the
tile keeps z's high word, and form the odd counter of each even-odd pair from
the even one's first product when bit 30 of z does not change either; a tile
across a multiple of 2^30 (or 2^32) takes the general 64-bit form.  Here every
method's single stream starts a few counters before a multiple of 2^30 and of
2^32, with the first z even and odd, so that its first tile takes the general
form and the next ones the paired forms of both parities, and is compared with
the oracle value by value (the rejection methods with their consumed count).  B3 runs in FP64 too, where
a lane takes one pair and the lanes' counter parities alternate.
"""
import pytest

import oracle as O
from gpu_util import assert_close, dev, host, run
from paper_1004_3105_amd import binding as nb

pytestmark = pytest.mark.gpu

GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1
ORACLE = {"b1": O.b1, "polar": O.polar, "polar2": O.polar2, "b3": O.b3, "ratio": O.ratio, "b2": O.b2}


def seed_for(boundary_bits: int, before: int) -> int:
    """A seed whose first z = seed + gamma lies `before` counters under a
    multiple of 2^boundary_bits (offset 0)."""
    return ((1 << boundary_bits) * 3 - before - GAMMA) & M64


@pytest.mark.parametrize("method", ["b1", "polar", "polar2", "b3", "ratio", "b2"])
@pytest.mark.parametrize("bits,before", [(30, 100), (30, 101), (32, 6), (32, 7), (31, 4096), (30, 1)])
def test_stream_across_hash_mode_boundaries(method, bits, before):
    dev()
    seed = seed_for(bits, before)
    n = (1 << 16) + 3
    dtypes = [nb.NRNG_F32] + ([nb.NRNG_F64] if method == "b3" else [])
    for dtype in dtypes:
        z, used = run(method, seed, 0, n, dtype, 0.25, 1.5, with_consumed=True)
        ref, uref = ORACLE[method](seed, 0, n, 0.25, 1.5)
        if method in ("polar", "polar2", "ratio"):
            assert used == uref
        extra = None
        if method == "b2" and dtype == nb.NRNG_F32:
            from helpers import b2_f32_extra
            pairs, _ = O.b2(seed, 0, 2 * ((n + 1) // 2), 0.25, 1.5)
            extra = b2_f32_extra(pairs, 0.25, n)
        assert_close(host(z), ref, dtype, 0.25, 1.5, what="%s across 2^%d" % (method, bits),
                     poly=method in ("polar2", "b3"), extra=extra)
