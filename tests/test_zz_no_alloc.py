"""The allocation-free Polar entry point, nrng_polar_noalloc, through the C
ABI: calls in a row on one device, each smaller than the one before (the
largest at the 2^26 maximum of its fixed scratch), each equal bit for bit to
nrng_polar's output with the same arguments, with the same consumed count,
and the smallest also against the oracle (Algorithm P, Section 2)."""
import pytest
import torch

import oracle as O
from gpu_util import TDT, NAME, assert_close, case, dev, host, u64
from paper_1004_3105_amd import binding as nb

pytestmark = pytest.mark.gpu

CALLS = [  # (seed, offset, n, mu, sigma), n decreasing
    (7, 0, 1 << 26, 0.0, 1.0),
    (7, 12345, (1 << 22) + 3, 0.5, 2.0),
    (11, 99, 100003, -1.0, 0.75),
]


@pytest.mark.parametrize("dtype", [nb.NRNG_F32, nb.NRNG_F64, nb.NRNG_BF16])
def test_noalloc_polar_equals_polar_in_decreasing_calls(dtype):
    d = dev()
    for seed, off, n, mu, sg in CALLS:
        ref = torch.full((n,), float("nan"), dtype=TDT[dtype], device=d)
        got = torch.full((n,), float("nan"), dtype=TDT[dtype], device=d)
        c_ref = torch.zeros(1, dtype=torch.int64, device=d)
        c_got = torch.zeros(1, dtype=torch.int64, device=d)
        case("polar_noalloc", NAME[dtype], "seed", seed, "offset", off, "n", n)
        nb.nrng_polar(seed, off, n, mu, sg, ref, dtype, None, c_ref)
        nb.nrng_polar_noalloc(seed, off, n, mu, sg, got, dtype, None, c_got)
        torch.cuda.synchronize()
        assert not torch.isnan(got).any(), n
        assert torch.equal(got, ref), n
        assert int(u64(c_got)[0]) == int(u64(c_ref)[0]), n
    seed, off, n, mu, sg = CALLS[-1]
    z_ref, used = O.polar(seed, off, n, mu, sg)
    assert int(u64(c_got)[0]) == used
    assert_close(host(got), z_ref, dtype, mu, sg, what="polar_noalloc vs oracle")


def test_noalloc_rejects_sizes_beyond_its_scratch():
    """n = 2^26 + 1 is refused with NRNG_ERANGE before any launch."""
    out = torch.empty(16, dtype=torch.float32, device=dev())
    with pytest.raises(nb.NrngError) as e:
        nb.nrng_polar_noalloc(1, 0, (1 << 26) + 1, 0.0, 1.0, out.data_ptr(), nb.NRNG_F32)
    assert e.value.status == nb.NRNG_ERANGE
