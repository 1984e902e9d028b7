"""Writes nrng_p2_poly.hpp: the polynomial coefficients of method P2's
radius factor for the HIP kernels.

Method P2 (Brent 1993, Section 4) evaluates g(s) = sqrt(-ln(1 - s) / s) for
0 <= s <= 8/9 through the change of variable v = (6 s - 4) / (4 - 3 s) of
Section 3 (rho = 1), which maps [0, 8/9] onto [-1, 1], and a polynomial h(v)
obtained by truncating the Chebyshev series of h(v) = g(s(v)) on [-1, 1].

Here the Chebyshev coefficients c_k = (2/pi) int_0^pi h(cos t) cos(k t) dt
are computed by mpmath quadrature at 60 significant digits, the truncated
series sum_{k<=d} c_k T_k(v) is expanded into powers of v in the same
precision, and the monomial coefficients are rounded once to the kernel's
arithmetic type:

    degree 15 in double precision (the degree the paper uses, truncation
        error about 1.5e-11 on [-1, 1]), for FP64 output;
    degree 9 in single precision (truncation error about 6e-8, below the
        rounding of an FP32 result of magnitude 1 to 1.6), for FP32, BF16 and
        FP16 output.

Run: python gen_p2_poly.py  (rewrites nrng_p2_poly.hpp beside this file).
"""
import os

import mpmath as mp
import numpy as np

mp.mp.dps = 60
HERE = os.path.dirname(os.path.abspath(__file__))


def g(s):
    if s == 0:
        return mp.mpf(1)
    return mp.sqrt(-mp.log1p(-s) / s)


def h(v):
    # inverse of v = (6 s - 4) / (4 - 3 s): s = 4 (v + 1) / (6 + 3 v)
    return g(4 * (v + 1) / (6 + 3 * v))


def cheb_coeffs(deg):
    c = []
    for k in range(deg + 1):
        ck = 2 / mp.pi * mp.quad(lambda t: h(mp.cos(t)) * mp.cos(k * t), [0, mp.pi / 2, mp.pi])
        c.append(ck / 2 if k == 0 else ck)
    return c


def cheb_to_monomial(c):
    # T_0 = 1, T_1 = v, T_{k+1} = 2 v T_k - T_{k-1}, as coefficient lists
    n = len(c)
    T = [[mp.mpf(1)] + [mp.mpf(0)] * (n - 1), [mp.mpf(0), mp.mpf(1)] + [mp.mpf(0)] * (n - 2)]
    for k in range(2, n):
        t = [mp.mpf(0)] * n
        for i in range(n - 1):
            t[i + 1] += 2 * T[k - 1][i]
        for i in range(n):
            t[i] -= T[k - 2][i]
        T.append(t)
    a = [mp.mpf(0)] * n
    for k in range(n):
        for i in range(n):
            a[i] += c[k] * T[k][i]
    return a


def max_error(a_rounded, dtype, deg):
    """Largest |horner(v) - g(s)| over a dense grid of s in [0, 8/9], with the
    polynomial evaluated in dtype (numpy) from the rounded coefficients."""
    s = np.linspace(0.0, 8.0 / 9.0, 20001)
    v = ((6 * s - 4) / (4 - 3 * s)).astype(dtype)
    p = np.full_like(v, a_rounded[deg])
    for i in range(deg - 1, -1, -1):
        p = p * v + dtype(a_rounded[i])
    ref = np.array([float(g(mp.mpf(float(x)))) for x in s])
    return float(np.max(np.abs(p.astype(np.float64) - ref)))


def main():
    out = []
    for deg, ctype, np_t, name, fmt in ((15, "double", np.float64, "kP2PolyF64", "%.17g"),
                                        (9, "float", np.float32, "kP2PolyF32", "%.9gf")):
        a = cheb_to_monomial(cheb_coeffs(deg))
        ar = [np_t(float(x)) for x in a]
        err = max_error(ar, np_t, deg)
        body = ",\n    ".join(fmt % float(x) for x in ar)
        out.append("// degree %d, coefficients of v^0 .. v^%d; max |h - g| over [0, 8/9] with\n"
                   "// %s evaluation by Horner's rule: %.2e\n"
                   "constexpr int %sDeg = %d;\n"
                   "__device__ constexpr %s %s[%d] = {\n    %s};\n"
                   % (deg, deg, ctype, err, name, deg, ctype, name, deg + 1, body))
    text = ("// nrng_p2_poly.hpp -- written by gen_p2_poly.py; do not edit.\n"
            "// Monomial coefficients of h(v), the truncated Chebyshev series on [-1, 1]\n"
            "// of g(s) = sqrt(-ln(1 - s) / s) under v = (6 s - 4) / (4 - 3 s)\n"
            "// (method P2, Brent 1993, Sections 3 and 4).\n"
            "#pragma once\n\nnamespace nrng {\n\n" + "\n".join(out) + "\n}  // namespace nrng\n")
    with open(os.path.join(HERE, "nrng_p2_poly.hpp"), "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
