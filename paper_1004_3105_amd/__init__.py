"""Normal random deviates on AMD Instinct MI355X (gfx950).

Box-Muller (Algorithm B1) and the Polar method (Algorithm P) of Brent,
"Fast Normal Random Number Generators for Vector Processors" (1993),
Section 2, over a counter-based SplitMix64 uniform stream, as hand-written
HIP kernels behind the C ABI of libnrng.so (include/nrng.h).

``binding`` mirrors the C entry points one to one; the helpers below only
allocate the output tensor with torch and call them.  Nothing here computes
deviates on the host.
"""
from __future__ import annotations

from . import binding
from .binding import (NRNG_BF16, NRNG_F16, NRNG_F32, NRNG_F64, NRNG_METHOD_B1, NRNG_METHOD_POLAR,  # noqa: F401
                      NrngError)

__all__ = ["binding", "normal", "torch_dtype", "NrngError", "NRNG_F64", "NRNG_F32", "NRNG_BF16", "NRNG_F16",
           "NRNG_METHOD_B1", "NRNG_METHOD_POLAR"]


def torch_dtype(dtype: int):
    import torch
    return {NRNG_F64: torch.float64, NRNG_F32: torch.float32, NRNG_BF16: torch.bfloat16,
            NRNG_F16: torch.float16}[dtype]


def normal(n: int, method: str = "polar", dtype: int = NRNG_F32, seed: int = 0, offset: int = 0,
           mu: float = 0.0, sigma: float = 1.0, device=None, stream=None, consumed: bool = False):
    """Allocate a tensor of n deviates on the GPU and fill it.

    With consumed=True (Polar only), also return a one-element uint64 device
    tensor (int64 bits of the uint64 count) holding the number of uniforms
    consumed."""
    import torch
    dev = torch.device("cuda") if device is None else torch.device(device)
    out = torch.empty(n, dtype=torch_dtype(dtype), device=dev)
    if method == "b1":
        binding.nrng_boxmuller(seed, offset, n, mu, sigma, out, dtype, stream)
        return out
    if method != "polar":
        raise ValueError("method must be 'b1' or 'polar'")
    cons = torch.zeros(1, dtype=torch.int64, device=dev) if consumed else None
    binding.nrng_polar(seed, offset, n, mu, sigma, out, dtype, stream, cons)
    return (out, cons) if consumed else out
