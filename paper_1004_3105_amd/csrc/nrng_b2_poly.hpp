// nrng_b2_poly.hpp -- written by gen_b2_poly.py; do not edit.
// Method B2 (Brent 1993, Section 3): sin y ~= y (s1 + t (s3 + t (s5 + t s7))) and
// cos y ~= c0 + t (c2 + t (c4 + t c6)), t = y^2, |y| <= pi/16: the Chebyshev series
// of sin(y)/y and cos(y) in t on [0, (pi/16)^2], truncated after T_3.
// kB2Sin* = {s1, s3, s5, s7}, kB2Cos* = {c0, c2, c4, c6}.
#pragma once

namespace nrng {

// F64: max |error| of sin 16y and cos 16y after the four doublings,
// evaluated in double over v in [0, 1): 1.90e-12
__device__ constexpr double kB2SinF64[4] = {0x1.ffffffffffe54p-1, -0x1.55555553fa564p-3, 0x1.11110614302b0p-7, -0x1.9fa7fc66d53eep-13};
__device__ constexpr double kB2CosF64[4] = {0x1.ffffffffff0f4p-1, -0x1.fffffff9e6c5cp-2, 0x1.55553c9d47e9fp-5, -0x1.6b967f2449fa3p-10};

// F32: max |error| of sin 16y and cos 16y after the four doublings,
// evaluated in float over v in [0, 1): 6.83e-07
__device__ constexpr float kB2SinF32[4] = {0x1.0000000000000p+0f, -0x1.5555560000000p-3f, 0x1.1111060000000p-7f, -0x1.9fa7fc0000000p-13f};
__device__ constexpr float kB2CosF32[4] = {0x1.0000000000000p+0f, -0x1.0000000000000p-1f, 0x1.55553c0000000p-5f, -0x1.6b96800000000p-10f};

}  // namespace nrng
