"""The FP64 oracle against its pins (CPU only)."""
import pytest

import oracle_pins as P


@pytest.mark.parametrize("check", P.ALL_CHECKS, ids=lambda f: f.__name__)
def test_oracle_pin(check):
    check()


def test_lattice_counts_known_values():
    # independent closed-form cross-check of the lattice counter used above:
    # sum over x of (2 isqrt(R^2 - 1 - x^2) + 1), minus the origin, for grids
    # small enough that no y is clipped by the box.
    import math
    for b in range(2, 9):
        R2 = 1 << (2 * b - 2)
        h = 1 << (b - 1)
        tot = sum(2 * math.isqrt(R2 - 1 - x * x) + 1 for x in range(-h + 1, h)) - 1
        assert P.lattice_count(b) == tot
    assert [P.lattice_count(b) for b in range(1, 9)] == [0, 8, 44, 192, 792, 3204, 12848, 51428]
