"""Writes nrng_b2_poly.hpp: the coefficients of method B2's inline sine and
cosine for the HIP kernels.

Method B2 (Brent 1993, Section 3) is Algorithm B1 with sin and cos of the
angle 2 pi v - pi computed from y = (2 pi v - pi)/16, |y| <= pi/16, by the
odd polynomial s1 y + s3 y^3 + s5 y^5 + s7 y^7, the even polynomial
c0 + c2 y^2 + c4 y^4 + c6 y^6 and four angle doublings.  The paper does not
print the coefficients.  They are taken as the Chebyshev series of sin(y)/y
and of cos(y), as functions of t = y^2 on [0, (pi/16)^2], truncated after
T_3, in powers of t.

Here the Chebyshev coefficients a_k = (2/pi) int_0^pi f(t(cos th)) cos(k th) dth,
t(x) = (pi/16)^2 (x + 1)/2, are computed by mpmath quadrature at 60
significant digits, the truncated series is expanded into powers of t in the
same precision, and each coefficient is rounded once to double (FP64 output)
and to single precision (FP32, BF16 and FP16 output).

Run: python gen_b2_poly.py  (rewrites nrng_b2_poly.hpp beside this file).
"""
import os

import mpmath as mp
import numpy as np

mp.mp.dps = 60
HERE = os.path.dirname(os.path.abspath(__file__))
TMAX = (mp.pi / 16) ** 2


def sin_over_y(t):
    if t == 0:
        return mp.mpf(1)
    y = mp.sqrt(t)
    return mp.sin(y) / y


def cos_y(t):
    return mp.cos(mp.sqrt(t))


def powers_of_t(f):
    """Truncated (T_0 .. T_3) Chebyshev series of f on [0, TMAX], in powers of t."""
    a = []
    for k in range(4):
        ak = 2 / mp.pi * mp.quad(lambda th: f(TMAX * (mp.cos(th) + 1) / 2) * mp.cos(k * th), [0, mp.pi])
        a.append(ak / 2 if k == 0 else ak)
    # sum a_k T_k(x) = p0 + p1 x + p2 x^2 + p3 x^3
    p = [a[0] - a[2], a[1] - 3 * a[3], 2 * a[2], 4 * a[3]]
    # x = (2 / TMAX) t - 1
    al = 2 / TMAX
    m = []
    for i in range(4):
        m.append(al ** i * sum(p[j] * mp.binomial(j, i) * (-1) ** (j - i) for j in range(i, 4)))
    return m


def doubled_error(s, c, dtype):
    """Largest |sin 16y - approx|, |cos 16y - approx| over a dense grid of
    v in [0, 1), evaluated in dtype from the rounded coefficients (the FP64
    kernel's order of operations; numpy rounds every operation)."""
    v = np.linspace(0.0, 1.0, 400001)[:-1]
    th = 2 * np.pi * v - np.pi
    y = (th / 16).astype(dtype)
    t = y * y
    sv = y * (s[0] + t * (s[1] + t * (s[2] + t * s[3])))
    cv = c[0] + t * (c[1] + t * (c[2] + t * c[3]))
    two, one = dtype(2), dtype(1)
    for _ in range(4):
        s2 = two * sv * cv
        cv = one - two * sv * sv
        sv = s2
    return float(max(np.max(np.abs(sv - np.sin(th))), np.max(np.abs(cv - np.cos(th)))))


def main():
    ms, mc = powers_of_t(sin_over_y), powers_of_t(cos_y)
    out = []
    # exact hexadecimal literals: the rounded values themselves, whatever the printing precision
    for ctype, np_t, suffix, sfx in (("double", np.float64, "F64", ""), ("float", np.float32, "F32", "f")):
        s = [np_t(float(x)) for x in ms]
        c = [np_t(float(x)) for x in mc]
        err = doubled_error(s, c, np_t)
        out.append("// %s: max |error| of sin 16y and cos 16y after the four doublings,\n"
                   "// evaluated in %s over v in [0, 1): %.2e\n"
                   "__device__ constexpr %s kB2Sin%s[4] = {%s};\n"
                   "__device__ constexpr %s kB2Cos%s[4] = {%s};\n"
                   % (suffix, ctype, err, ctype, suffix, ", ".join(float(x).hex() + sfx for x in s),
                      ctype, suffix, ", ".join(float(x).hex() + sfx for x in c)))
    text = ("// nrng_b2_poly.hpp -- written by gen_b2_poly.py; do not edit.\n"
            "// Method B2 (Brent 1993, Section 3): sin y ~= y (s1 + t (s3 + t (s5 + t s7))) and\n"
            "// cos y ~= c0 + t (c2 + t (c4 + t c6)), t = y^2, |y| <= pi/16: the Chebyshev series\n"
            "// of sin(y)/y and cos(y) in t on [0, (pi/16)^2], truncated after T_3.\n"
            "// kB2Sin* = {s1, s3, s5, s7}, kB2Cos* = {c0, c2, c4, c6}.\n"
            "#pragma once\n\nnamespace nrng {\n\n" + "\n".join(out) + "\n}  // namespace nrng\n")
    with open(os.path.join(HERE, "nrng_b2_poly.hpp"), "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
