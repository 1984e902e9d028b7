// nrng_p2_poly.hpp -- written by gen_p2_poly.py; do not edit.
// Monomial coefficients of h(v), the truncated Chebyshev series on [-1, 1]
// of g(s) = sqrt(-ln(1 - s) / s) under v = (6 s - 4) / (4 - 3 s)
// (method P2, Brent 1993, Sections 3 and 4).
#pragma once

namespace nrng {

// degree 15, coefficients of v^0 .. v^15; max |h - g| over [0, 8/9] with
// double evaluation by Horner's rule: 1.51e-11
constexpr int kP2PolyF64Deg = 15;
__device__ constexpr double kP2PolyF64[16] = {
    1.2837127533005859,
    0.2633146634418313,
    0.0018012621610910982,
    0.019510673659028033,
    0.00046001010841604037,
    0.0027179094762193653,
    0.00010548884506850869,
    0.00046038556687944134,
    2.3398026173703506e-05,
    8.4177554298281202e-05,
    6.3568180845116704e-06,
    1.9708859673353308e-05,
    2.3612730210796403e-07,
    7.5611402943227693e-07,
    8.0008248942255221e-07,
    2.0307960008223673e-06};

// degree 9, coefficients of v^0 .. v^9; max |h - g| over [0, 8/9] with
// float evaluation by Horner's rule: 1.65e-07
constexpr int kP2PolyF32Deg = 9;
__device__ constexpr float kP2PolyF32[10] = {
    1.28371274f,
    0.263315022f,
    0.001800225f,
    0.019503722f,
    0.000467992591f,
    0.00275541027f,
    8.447445e-05f,
    0.000379614939f,
    4.48145656e-05f,
    0.000156500668f};

}  // namespace nrng
