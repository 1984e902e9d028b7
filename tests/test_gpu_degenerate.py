"""Degenerate parameters through the C ABI: sigma = 0 gives exactly mu for
every method and output type (the FP32 radius forms fold sigma into their
constants, and Polar's rare FP64 radius multiplies by it), and the rejection
methods still consume what the oracle consumes, since sigma does not enter
their acceptance tests."""
import pytest
import torch

import oracle as O
from gpu_util import run
from paper_1004_3105_amd import binding as nb

pytestmark = pytest.mark.gpu

COUNTED = {"polar": O.polar, "polar2": O.polar2, "ratio": O.ratio}
N = (1 << 22) + 7   # enough pairs that Polar meets s < 2^-20 (its FP64 branch)


@pytest.mark.parametrize("method", ["b1", "polar", "polar2", "b3", "ratio", "b2"])
@pytest.mark.parametrize("dtype", [nb.NRNG_F64, nb.NRNG_F32, nb.NRNG_BF16, nb.NRNG_F16])
def test_sigma_zero_gives_exactly_mu(method, dtype):
    z, used = run(method, 11, 3, N, dtype, 2.5, 0.0, with_consumed=True)
    assert torch.all(z == 2.5), int((z != 2.5).sum())
    if method in COUNTED:
        _, used_ref = COUNTED[method](11, 3, N)
        assert used == used_ref
