"""Pins of the FP64 oracle to facts outside itself.

Each check raises AssertionError on failure.  They are run directly by
test_oracle_pins.py and, against deliberately broken CPU builds of the
oracle, by test_oracle_mutants.py (which requires every planted mistake to
trip at least one of them).

What pins what:
  * the SplitMix64 check sequence (published test vector) pins the uniform
    generator, and the definitions u = (k >> 11) 2^-53 and X = int32(k >> 32)
    are checked against those published words;
  * closed-form values of Algorithms B1 and P (Section 2) pin the
    transforms, with inputs chosen so that swapping u and v, sin and cos, x
    and y, dropping a factor of 2 or of s, or using u instead of 1 - u all
    change the result;
  * a brute-force lattice count (integer arithmetic written here) pins the
    acceptance predicate, including the boundary circle S = 2^62;
  * the acceptance rate pi/4, the uniformity of the accepted s and of the
    polar angle, and moments / KS against the normal CDF pin the stream
    composition statistically;
  * SciPy pins the oracle's statistics routines;
  * method P2 (Section 4): the paper's error bound of its degree-15
    polynomial (below 2e-11 on [-1, 1]) against g(s) = sqrt(-ln(1-s)/s)
    computed here from the closed form, closed-form values on both sides of
    the split at s = 8/9, the lattice count with the origin accepted, the
    identity z_P2 = z_P sqrt(ln(1 - s)/ln(s)) pair by pair against the Polar
    stream, and -ln(1 - s) = (zx^2 + zy^2)/2 being exponential(1);
  * method B3 (Section 3): closed-form values (max rather than min, the
    order cos then sin, the shift by -pi, both sides of 8/9), the whole
    stream pair by pair against sqrt(-2 log1p(-m^2)) (cos t, sin t)
    computed here, 3 uniforms per pair, and the distribution;
  * method B2 (Section 3): closed-form values (the angle 2 pi v - pi, the
    factor 16, the order sin then cos), the paper's error bound on the inline
    sine and cosine against the library (which Taylor coefficients would
    miss), the error's orthogonality to T_0 .. T_3 (the truncated Chebyshev
    series), B2 == -B1 pair by pair, and the stream and distribution;
  * Algorithm R (Section 5): closed-form accept/reject cases on both sides
    of the curve x^2 = -4 ln(1 - u), the acceptance rate sqrt(pi e)/4 (the
    2.74 uniforms per normal the section states), the stream's composition,
    and the distribution of the accepted x.
"""
from __future__ import annotations

import math

import numpy as np

import oracle as O
from helpers import closed_form, golden_rows, stat_bounds, ulp_dist64

GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def _published():
    rows = []
    import os
    from helpers import GOLDEN
    with open(os.path.join(GOLDEN, "splitmix64_check.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                i, v = line.split()
                rows.append((int(i), int(v, 16)))
    return rows


# ------------------------------------------------------------------ uniforms
def check_splitmix_published():
    for i, v in _published():
        got = O.splitmix64((i * GAMMA) & M64)
        assert got == v, (i, hex(got), hex(v))


def check_stream_definitions():
    pub = dict(_published())
    # u_i = (k >> 11) 2^-53 and X_i = int32(k >> 32) with k = splitmix64(seed + offset + i)
    for i in range(4):
        seed = (i * GAMMA) & M64
        u = O.uniforms(seed, 0, 1)[0]
        assert u == (pub[i] >> 11) * 2.0**-53, i
        X = int(O.int32s(seed, 0, 1)[0])
        hi = pub[i] >> 32
        assert X == (hi - (1 << 32) if hi >= (1 << 31) else hi), i
        assert int(O.hashes(seed, 0, 1)[0]) == pub[i]
    # the counter is seed + offset + i, wrapping mod 2^64
    assert int(O.hashes(M64, 0, 2)[1]) == pub[0]
    assert int(O.hashes(M64 - 5, 3, 4)[3]) == pub[0]
    a = O.hashes(12345, 678, 16)
    b = O.hashes(12345 + 678, 0, 16)
    c = O.hashes(0, 12345 + 678, 16)
    assert np.array_equal(a, b) and np.array_equal(a, c)
    assert np.all(O.uniforms(3, 0, 4096) < 1.0) and np.all(O.uniforms(3, 0, 4096) >= 0.0)


# ------------------------------------------------------------------ B1
def check_b1_hand():
    rows = golden_rows("b1_hand_values.txt")
    u = np.array([closed_form(r[0]) for r in rows])
    v = np.array([closed_form(r[1]) for r in rows])
    out = O.b1_uv(u, v).reshape(-1, 2)
    for k, r in enumerate(rows):
        for c in range(2):
            want = closed_form(r[2 + c])
            budget = int(r[4])
            got = out[k, c]
            if want == 0.0:
                assert abs(got) <= 1e-15, (r, c, got)
            else:
                assert ulp_dist64([got], [want])[0] <= budget, (r, c, got, want)
    # mu and sigma enter as sigma * (...) + mu
    out2 = O.b1_uv(u, v, mu=-3.0, sigma=2.5).reshape(-1, 2)
    assert np.allclose(out2, -3.0 + 2.5 * out, rtol=0, atol=1e-14)


def check_b1_words_definition():
    # u = (w >> 11) 2^-53 for the first word of a pair, v likewise for the second
    w = np.array([1 << 63, 1 << 61, 3 << 62, 1 << 62, 0, (12345 << 11) + 7, ((1 << 53) - 1) << 11, 1 << 62],
                 dtype=np.uint64)
    got = O.b1_words(w)
    want = O.b1_uv([0.5, 0.75, 0.0, 1 - 2.0**-53], [0.125, 0.25, 12345 * 2.0**-53, 0.25])
    assert np.array_equal(got, want)


def check_b1_composition():
    seed, off, n = 0x5EED, 1000, 4097
    z, used = O.b1(seed, off, n)
    assert used == 2 * ((n + 1) // 2)
    u = O.uniforms(seed, off, used)
    ref = O.b1_uv(u[0::2], u[1::2])[:n]
    assert np.array_equal(z, ref)
    # raw words give the same stream
    assert np.array_equal(O.b1_words(O.hashes(seed, off, used))[:n], ref)
    # concatenation: the stream from offset off + 2k continues the same values
    z2, _ = O.b1(seed, off + 2 * 100, n - 200)
    assert np.array_equal(z2, z[200:])
    # mu, sigma
    zs, _ = O.b1(seed, off, n, mu=1.5, sigma=0.5)
    assert np.allclose(zs, 1.5 + 0.5 * z, rtol=0, atol=1e-14)


# ------------------------------------------------------------------ Polar
def check_polar_hand():
    rows = golden_rows("polar_hand_values.txt")
    xy = np.array([[int(r[0]), int(r[1])] for r in rows], dtype=np.int64).astype(np.int32)
    out, masks, a = O.polar_xy(xy)
    acc = [int(r[2]) for r in rows]
    assert a == sum(acc)
    bits = [(int(masks[j // 64]) >> (j % 64)) & 1 for j in range(len(rows))]
    assert bits == acc, (bits, acc)
    vals = out.reshape(-1, 2)
    k = 0
    for r in rows:
        if r[2] == "0":
            assert not O.polar_accept(int(r[0]), int(r[1]))
            continue
        for c in range(2):
            want = closed_form(r[3 + c])
            got = vals[k, c]
            if want == 0.0:
                assert got == 0.0, (r, got)
            else:
                assert ulp_dist64([got], [want])[0] <= 4, (r, c, got, want)
        k += 1
    out2, _, _ = O.polar_xy(xy, mu=2.0, sigma=3.0)
    assert np.allclose(out2, 2.0 + 3.0 * out, rtol=0, atol=1e-13)


def lattice_count(b: int) -> int:
    """#{(x, y) in [-2^(b-1), 2^(b-1))^2 : 0 < x^2 + y^2 < 2^(2b-2)}, by
    counting, for each x, the integers y with y^2 < R^2 - x^2."""
    R2 = 1 << (2 * b - 2)
    h = 1 << (b - 1)
    tot = 0
    for x in range(-h, h):
        rem = R2 - 1 - x * x
        if rem < 0:
            continue
        m = math.isqrt(rem)                 # |y| <= m
        lo, hi = max(-m, -h), min(m, h - 1)
        tot += hi - lo + 1
    return tot - 1                          # drop the origin


def check_polar_lattice(bmax: int = 10):
    for b in range(1, bmax + 1):
        h = 1 << (b - 1)
        g = np.arange(-h, h, dtype=np.int64)
        X, Y = np.meshgrid(g, g, indexing="ij")
        shift = 32 - b
        xy = np.stack([X.ravel() << shift, Y.ravel() << shift], axis=1).astype(np.int32)
        _, masks, a = O.polar_xy(xy)
        assert a == lattice_count(b), (b, a, lattice_count(b))
    # the four points on the circle S = 2^62 and their neighbours
    R = 1 << 31
    for (x, y, acc) in [(-R, 0, 0), (0, -R, 0), (-R, -R, 0), (R - 1, 0, 1), (0, R - 1, 1), (-R + 1, 0, 1),
                        (-R, 1, 0), (0, 0, 0), (1, 0, 1), (0, 1, 1)]:
        assert O.polar_accept(x, y) == bool(acc), (x, y)
    # random points against exact Python integers
    g = np.random.Generator(np.random.PCG64(99))
    pts = g.integers(-R, R, (20000, 2))
    _, masks, a = O.polar_xy(pts.astype(np.int32))
    want = [(0 < int(x) * int(x) + int(y) * int(y) < (1 << 62)) for x, y in pts]
    bits = np.unpackbits(masks.view(np.uint8), bitorder="little")[:len(want)].astype(bool)
    assert np.array_equal(bits, np.array(want))


def check_polar_composition():
    seed, off, n = 7, 12, 20001
    z, used = O.polar(seed, off, n)
    ncand = used // 2
    xy = O.int32s(seed, off, used)
    ref, masks, a = O.polar_xy(xy)
    assert a == (n + 1) // 2
    # the last candidate consumed is the one that supplied the last value
    assert (int(masks[(ncand - 1) // 64]) >> ((ncand - 1) % 64)) & 1 == 1
    assert np.array_equal(z, ref[:n])
    # trace and count agree with the mask of the explicit path
    tm, tp, ta = O.polar_trace(seed, off, ncand)
    assert np.array_equal(tm, masks) and ta == a
    pc = np.concatenate([[0], np.cumsum([bin(int(m)).count("1") for m in masks])])[:-1]
    assert np.array_equal(tp.astype(np.int64), pc)
    assert O.polar_count(seed, off, ncand) == a
    # a window of the stream reproduces the same slice
    j0 = 1000
    w = O.polar_window(seed, off, j0, 3000)
    before = O.polar_count(seed, off, j0)
    assert np.array_equal(w, ref[2 * before: 2 * before + w.size])
    # concatenation: restarting at the consumed offset continues the stream
    z1, used1 = O.polar(seed, off, 1000)
    z2, used2 = O.polar(seed, off + used1, n - 1000)
    assert np.array_equal(np.concatenate([z1, z2]), z) and used1 + used2 == used


def check_polar_accept_rate(ncand: int = 1 << 21):
    a = O.polar_count(0xACCE, 0, ncand)
    p = math.pi / 4
    assert abs(a / ncand - p) < 5 * math.sqrt(p * (1 - p) / ncand), a / ncand


def check_polar_s_uniform(ncand: int = 1 << 19):
    from scipy import stats
    xy = O.int32s(0x5, 0, 2 * ncand).astype(np.int64).reshape(-1, 2)
    S = xy[:, 0] ** 2 + xy[:, 1] ** 2          # exact in int64 except at S = 2^63
    _, masks, a = O.polar_xy(xy.astype(np.int32))
    bits = np.unpackbits(masks.view(np.uint8), bitorder="little")[:ncand].astype(bool)
    s = S[bits].astype(np.float64) * 2.0**-62
    assert s.size == a
    assert stats.kstest(s, "uniform").statistic < 1.95 / math.sqrt(a)


def _dist_checks(z: np.ndarray):
    from scipy import stats
    N = z.size
    bd = stat_bounds(N)
    assert abs(z.mean()) < bd["mean"], z.mean()
    assert abs(z.var() - 1) < bd["var"], z.var()
    assert abs(stats.skew(z)) < bd["skew"]
    assert abs(stats.kurtosis(z, fisher=False) - 3) < bd["kurt"]
    assert stats.kstest(z, "norm").statistic < bd["ks"]
    r = np.corrcoef(z[:-1], z[1:])[0, 1]
    assert abs(r) < 5 / math.sqrt(N)


def check_b1_distribution(n: int = 1 << 20):
    z, _ = O.b1(1, 0, n)
    _dist_checks(z)
    # the angle of each pair is uniform: (x, y) = r (sin t, cos t)
    from scipy import stats
    ang = np.arctan2(z[0::2], z[1::2]) / (2 * math.pi) % 1.0
    assert stats.kstest(ang, "uniform").statistic < 1.95 / math.sqrt(ang.size)


def check_polar_distribution(n: int = 1 << 20):
    z, _ = O.polar(7, 0, n)
    _dist_checks(z)
    from scipy import stats
    ang = (np.arctan2(z[1::2], z[0::2]) / (2 * math.pi)) % 1.0
    assert stats.kstest(ang, "uniform").statistic < 1.95 / math.sqrt(ang.size)
    # r^2 / 2 = -ln s is exponential(1) for the accepted s
    e = 0.5 * (z[0::2] ** 2 + z[1::2] ** 2)
    assert stats.kstest(e, "expon").statistic < 1.95 / math.sqrt(e.size)


# ------------------------------------------------------------------ P2
def _g_closed(s: np.ndarray) -> np.ndarray:
    s = np.asarray(s, dtype=np.float64)
    out = np.ones_like(s)
    nz = s != 0
    out[nz] = np.sqrt(-np.log1p(-s[nz]) / s[nz])
    return out


def check_p2_poly_bound():
    # Section 3: the degree-15 truncation approximates h(v) = g(s) with
    # absolute error below 2e-11 on [-1, 1], and v = (6s - 4)/(4 - 3s) maps
    # [0, 8/9] onto [-1, 1]
    s = np.concatenate([np.linspace(0.0, 8.0 / 9.0, 4001), [1e-12, 1e-6, 0.5, 8.0 / 9.0]])
    v = (6 * s - 4) / (4 - 3 * s)
    assert abs(v[0] + 1) == 0 and abs(v[4000] - 1) < 1e-15
    h = np.array([O.p2_h(float(x)) for x in v])
    err = np.abs(h - _g_closed(s))
    assert err.max() < 2e-11, err.max()
    # g(u) = 1 + u/4 + ... near 0
    d = (O.p2_h(float((6 * 1e-4 - 4) / (4 - 3e-4))) - 1.0) / 1e-4
    assert abs(d - 0.25) < 1e-4, d
    # the coefficients decay like those of a function analytic inside the
    # ellipse through the singularities at v = +-2 (rate 2 - sqrt(3))
    c = O.p2_cheb(15)
    assert c[0] > 1.0 and np.all(np.abs(c[12:]) < 1e-8) and np.all(np.abs(c[4:]) < 1e-3)


def check_polar2_hand():
    rows = golden_rows("polar2_hand_values.txt")
    xy = np.array([[int(r[0]), int(r[1])] for r in rows], dtype=np.int64).astype(np.int32)
    out, masks, a = O.polar2_xy(xy)
    acc = [int(r[2]) for r in rows]
    assert a == sum(acc)
    bits = [(int(masks[j // 64]) >> (j % 64)) & 1 for j in range(len(rows))]
    assert bits == acc, (bits, acc)
    vals = out.reshape(-1, 2)
    k = 0
    for r in rows:
        if r[2] == "0":
            assert not O.polar2_accept(int(r[0]), int(r[1]))
            continue
        kind, amt = r[5].split(":")
        for c in range(2):
            want = closed_form(r[3 + c])
            got = vals[k, c]
            if kind == "abs" or want == 0.0:
                assert abs(got - want) <= float(amt), (r, c, got, want)
            else:
                assert ulp_dist64([got], [want])[0] <= int(amt), (r, c, got, want)
        k += 1
    out2, _, _ = O.polar2_xy(xy, mu=2.0, sigma=3.0)
    assert np.allclose(out2, 2.0 + 3.0 * out, rtol=0, atol=1e-13)


def check_polar2_lattice(bmax: int = 9):
    # P2 rejects only s >= 1, so its lattice count is Algorithm P's plus the origin
    for b in range(1, bmax + 1):
        h = 1 << (b - 1)
        g = np.arange(-h, h, dtype=np.int64)
        X, Y = np.meshgrid(g, g, indexing="ij")
        shift = 32 - b
        xy = np.stack([X.ravel() << shift, Y.ravel() << shift], axis=1).astype(np.int32)
        _, _, a = O.polar2_xy(xy)
        assert a == lattice_count(b) + 1, (b, a)
    R = 1 << 31
    for (x, y, acc) in [(-R, 0, 0), (0, -R, 0), (-R, -R, 0), (R - 1, 0, 1), (0, 0, 1), (1, 0, 1)]:
        assert O.polar2_accept(x, y) == bool(acc), (x, y)


def check_polar2_vs_polar():
    # same candidates, pairing, order and consumed count as Algorithm P (no
    # (0, 0) candidate occurs in these streams); pair by pair,
    # z_P2 = z_P sqrt(ln(1 - s) / ln(s)), with s from the stream's integers
    seed, off, n = 7, 12, 20001
    z2, used2 = O.polar2(seed, off, n)
    z1, used1 = O.polar(seed, off, n)
    assert used1 == used2
    xy = O.int32s(seed, off, used2).astype(np.int64).reshape(-1, 2)
    S = xy[:, 0] ** 2 + xy[:, 1] ** 2
    keep = (S > 0) & (S < (1 << 62))
    s = S[keep].astype(np.float64) * 2.0**-62
    ratio = np.sqrt(np.log1p(-s) / np.log(s))
    k = (n + 1) // 2
    want = (z1.reshape(-1) if n % 2 == 0 else np.append(z1, 0.0)).reshape(-1, 2) * ratio[:k, None]
    got = (z2 if n % 2 == 0 else np.append(z2, 0.0)).reshape(-1, 2)
    assert np.allclose(got, want, rtol=5e-10, atol=5e-10)
    # composition, as for Algorithm P: explicit candidates, windows, restarts
    ref, masks, a = O.polar2_xy(O.int32s(seed, off, used2))
    assert a == k and np.array_equal(z2, ref[:n])
    assert O.polar2_count(seed, off, used2 // 2) == a
    j0 = 1000
    w = O.polar2_window(seed, off, j0, 3000)
    before = O.polar2_count(seed, off, j0)
    assert np.array_equal(w, ref[2 * before: 2 * before + w.size])
    za, ua = O.polar2(seed, off, 1000)
    zb, ub = O.polar2(seed, off + ua, n - 1000)
    assert np.array_equal(np.concatenate([za, zb]), z2) and ua + ub == used2
    zs, _ = O.polar2(seed, off, n, mu=1.5, sigma=0.5)
    assert np.allclose(zs, 1.5 + 0.5 * z2, rtol=0, atol=1e-14)


def check_polar2_distribution(n: int = 1 << 20):
    z, _ = O.polar2(7, 0, n)
    _dist_checks(z)
    from scipy import stats
    ang = (np.arctan2(z[1::2], z[0::2]) / (2 * math.pi)) % 1.0
    assert stats.kstest(ang, "uniform").statistic < 1.95 / math.sqrt(ang.size)
    # (zx^2 + zy^2)/2 = -ln(1 - s), exponential(1) because 1 - s is uniform
    e = 0.5 * (z[0::2] ** 2 + z[1::2] ** 2)
    assert stats.kstest(e, "expon").statistic < 1.95 / math.sqrt(e.size)


# ------------------------------------------------------------------ B3
def check_b2_hand():
    rows = golden_rows("b2_hand_values.txt")
    u = np.array([closed_form(r[0]) for r in rows])
    v = np.array([closed_form(r[1]) for r in rows])
    out = O.b2_uv(u, v).reshape(-1, 2)
    for k, r in enumerate(rows):
        kind, amt = r[4].split(":")
        for c in range(2):
            want, got = closed_form(r[2 + c]), out[k, c]
            if kind == "abs" or want == 0.0:
                assert abs(got - want) <= float(amt), (r, c, got, want)
            else:
                assert ulp_dist64([got], [want])[0] <= int(amt), (r, c, got, want)
    w = np.stack([(np.round(u * 2.0**53).astype(np.uint64) << np.uint64(11)),
                  (np.round(v * 2.0**53).astype(np.uint64) << np.uint64(11))], axis=1).reshape(-1)
    assert np.array_equal(O.b2_words(w), out.reshape(-1))
    out2 = O.b2_uv(u, v, mu=-2.0, sigma=0.5)
    assert np.allclose(out2, -2.0 + 0.5 * out.reshape(-1), rtol=0, atol=1e-14)


def check_b2_bound():
    """Section 3 puts the error of B2's inline sine and cosine well below
    1e-10 in absolute terms; the degree-7/6 near-minimax polynomials with
    four doublings reach about 2e-12 (Taylor coefficients would give 2.4e-10).
    The coefficients are the truncated Chebyshev series: the error of each
    polynomial is orthogonal to T_0 .. T_3 under the Chebyshev weight
    (checked by Gauss-Chebyshev quadrature), and they are close to the Taylor
    coefficients of sin and cos."""
    v = np.concatenate([np.linspace(0.0, 1.0, 20001)[:-1], np.random.Generator(np.random.PCG64(21)).uniform(0.0, 1.0, 20000)])
    err = 0.0
    for x in v:
        sn, cs = O.b2_sincos(float(x))
        th = 2.0 * math.pi * float(x) - math.pi
        err = max(err, abs(sn - math.sin(th)), abs(cs - math.cos(th)))
    assert err < 1e-11, err
    assert err > 1e-13, err                    # an approximation, not the library
    s, c = O.b2_coef()
    taylor_s = [1.0, -1.0 / 6, 1.0 / 120, -1.0 / 5040]
    taylor_c = [1.0, -0.5, 1.0 / 24, -1.0 / 720]
    for got, tay in zip(list(s) + list(c), taylor_s + taylor_c):
        assert abs(got - tay) <= 2e-3 * abs(tay), (got, tay)
    tmax = (math.pi / 16) ** 2
    N = 64
    xj = np.cos(math.pi * (np.arange(N) + 0.5) / N)
    t = tmax * (xj + 1) / 2
    y = np.sqrt(t)
    for f, coef in ((np.sin(y) / y, s), (np.cos(y), c)):
        p = coef[0] + t * (coef[1] + t * (coef[2] + t * coef[3]))
        e = f - p
        for k in range(4):
            resid = abs(np.sum(e * np.cos(k * np.arccos(xj)))) / N
            assert resid < 1e-3 * np.max(np.abs(e)), (k, resid, np.max(np.abs(e)))


def check_b2_vs_b1():
    """B2's angle is B1's minus pi, on the same uniforms and radius, so pair
    k of B2 is pair k of B1 negated (about mu) up to the approximation."""
    seed, off, n = 0xB2, 5, 40000
    for mu, sigma in ((0.0, 1.0), (3.0, 0.25)):
        z2, c2 = O.b2(seed, off, n, mu, sigma)
        z1, c1 = O.b1(seed, off, n, mu, sigma)
        assert c1 == c2 == n
        d2, d1 = (z2 - mu).reshape(-1, 2), (z1 - mu).reshape(-1, 2)
        r = np.hypot(d1[:, 0], d1[:, 1])
        assert np.all(np.abs(d2 + d1) <= 4e-12 * r[:, None] + 1e-15), np.max(np.abs(d2 + d1))
        assert np.allclose(np.hypot(d2[:, 0], d2[:, 1]), r, rtol=1e-11, atol=0)


def check_b2_stream():
    # pair k takes uniforms 2k, 2k + 1; the stream equals the explicit-uniform
    # and explicit-word forms; n odd keeps the first value; restarting at
    # offset + consumed continues it
    seed, off, n = 0xB2B2, 33, 30001
    z, used = O.b2(seed, off, n)
    assert used == 2 * ((n + 1) // 2)
    u = O.uniforms(seed, off, used).reshape(-1, 2)
    ref = O.b2_uv(u[:, 0], u[:, 1])
    assert np.array_equal(z, ref[:n])
    assert np.array_equal(O.b2_words(O.hashes(seed, off, used))[:n], ref[:n])
    z1, c1 = O.b2(seed, off, 1000)
    z2, c2 = O.b2(seed, off + c1, n - 1000)
    assert np.array_equal(np.concatenate([z1, z2]), z) and c1 + c2 == used


def check_b2_distribution(n: int = 1 << 20):
    z, _ = O.b2(1, 0, n)
    _dist_checks(z)
    from scipy import stats
    ang = np.arctan2(z[0::2], z[1::2]) / (2 * math.pi) % 1.0
    assert stats.kstest(ang, "uniform").statistic < 1.95 / math.sqrt(ang.size)


def check_b3_hand():
    rows = golden_rows("b3_hand_values.txt")
    u1 = np.array([closed_form(r[0]) for r in rows])
    u2 = np.array([closed_form(r[1]) for r in rows])
    u3 = np.array([closed_form(r[2]) for r in rows])
    out = O.b3_u(u1, u2, u3).reshape(-1, 2)
    for k, r in enumerate(rows):
        kind, amt = r[5].split(":")
        for c in range(2):
            want, got = closed_form(r[3 + c]), out[k, c]
            if kind == "abs" or want == 0.0:
                assert abs(got - want) <= max(float(amt), 1e-15), (r, c, got, want)
            else:
                assert ulp_dist64([got], [want])[0] <= int(amt), (r, c, got, want)
    out2 = O.b3_u(u1, u2, u3, mu=2.0, sigma=3.0)
    assert np.allclose(out2, 2.0 + 3.0 * out.reshape(-1), rtol=0, atol=1e-13)


def check_b3_stream():
    # pair k takes uniforms 3k, 3k + 1, 3k + 2; the stream equals the
    # explicit-uniform and explicit-word forms; n odd keeps the first value;
    # restarting at offset + consumed continues it
    seed, off, n = 0xB3, 77, 30001
    z, used = O.b3(seed, off, n)
    P = (n + 1) // 2
    assert used == 3 * P
    u = O.uniforms(seed, off, used).reshape(-1, 3)
    ref = O.b3_u(u[:, 0], u[:, 1], u[:, 2])
    assert np.array_equal(z, ref[:n])
    assert np.array_equal(O.b3_words(O.hashes(seed, off, used))[:n], ref[:n])
    z1, c1 = O.b3(seed, off, 1000)
    z2, c2 = O.b3(seed, off + c1, n - 1000)
    assert np.array_equal(np.concatenate([z1, z2]), z) and c1 + c2 == used
    zs, _ = O.b3(seed, off, n, mu=-1.5, sigma=0.25)
    assert np.allclose(zs, -1.5 + 0.25 * z, rtol=0, atol=1e-14)
    # pair by pair against the closed form (the polynomial is within 2e-11
    # of g), computed here with NumPy's log1p, sin and cos
    m = np.maximum(u[:, 0], u[:, 1])
    r = np.sqrt(-2.0 * np.log1p(-(m * m)))
    t = 2.0 * np.pi * u[:, 2] - np.pi
    want = np.stack([r * np.cos(t), r * np.sin(t)], axis=1).reshape(-1)[:n]
    assert np.max(np.abs(z - want) / np.maximum(1.0, np.abs(want))) < 3e-11
    # and it is not the min(u1, u2) variant or the u3 -> u2 pairing
    m2 = np.minimum(u[:, 0], u[:, 1])
    r2 = np.sqrt(-2.0 * np.log1p(-(m2 * m2)))
    alt = np.stack([r2 * np.cos(t), r2 * np.sin(t)], axis=1).reshape(-1)[:n]
    assert np.max(np.abs(z - alt)) > 0.1


def check_b3_distribution(n: int = 1 << 20):
    z, _ = O.b3(3, 0, n)
    _dist_checks(z)
    from scipy import stats
    # the angle of (x, y) = r (cos t, sin t) is t = 2 pi u3 - pi
    ang = (np.arctan2(z[1::2], z[0::2]) / (2 * math.pi)) % 1.0
    assert stats.kstest(ang, "uniform").statistic < 1.95 / math.sqrt(ang.size)
    # (x^2 + y^2)/2 = -ln(1 - u) with u = max(u1, u2)^2 uniform
    e = 0.5 * (z[0::2] ** 2 + z[1::2] ** 2)
    assert stats.kstest(e, "expon").statistic < 1.95 / math.sqrt(e.size)


# ------------------------------------------------------------------ Algorithm R
def _word(u: float) -> int:
    return int(round(u * 2.0**53)) << 11


def check_ratio_hand():
    rows = golden_rows("ratio_hand_values.txt")
    w = np.array([_word(closed_form(r[c])) for r in rows for c in range(2)], dtype=np.uint64)
    out, masks, a = O.ratio_words(w)
    acc = [int(r[2]) for r in rows]
    assert a == sum(acc)
    bits = [(int(masks[j // 64]) >> (j % 64)) & 1 for j in range(len(rows))]
    assert bits == acc, (bits, acc)
    k = 0
    for r in rows:
        assert O.ratio_accept(closed_form(r[0]), closed_form(r[1])) == (r[2] == "1")
        if r[2] == "0":
            continue
        want, got = closed_form(r[3]), out[k]
        kind, amt = r[4].split(":")
        if kind == "abs" or want == 0.0:
            assert abs(got - want) <= float(amt), (r, got, want)
        else:
            assert ulp_dist64([got], [want])[0] <= int(amt), (r, got, want)
        k += 1
    out2, _, _ = O.ratio_words(w, mu=2.0, sigma=3.0)
    assert np.allclose(out2, 2.0 + 3.0 * out, rtol=0, atol=1e-13)


def check_ratio_rate(ncand: int = 1 << 21):
    a = O.ratio_count(0x5A7, 0, ncand)
    p = math.sqrt(math.pi * math.e) / 4
    assert abs(a / ncand - p) < 5 * math.sqrt(p * (1 - p) / ncand), a / ncand


def check_ratio_stream():
    seed, off, n = 0xA11, 9, 20001
    z, used = O.ratio(seed, off, n)
    ncand = used // 2
    w = O.hashes(seed, off, used)
    ref, masks, a = O.ratio_words(w)
    assert a == n and np.array_equal(z, ref)
    # the last candidate consumed supplied the last value
    assert (int(masks[(ncand - 1) // 64]) >> ((ncand - 1) % 64)) & 1 == 1
    tm, tp, ta = O.ratio_trace(seed, off, ncand)
    assert np.array_equal(tm, masks) and ta == a
    pc = np.concatenate([[0], np.cumsum([bin(int(m)).count("1") for m in masks])])[:-1]
    assert np.array_equal(tp.astype(np.int64), pc)
    assert O.ratio_count(seed, off, ncand) == a
    j0 = 1000
    win = O.ratio_window(seed, off, j0, 3000)
    before = O.ratio_count(seed, off, j0)
    assert np.array_equal(win, ref[before: before + win.size])
    z1, u1 = O.ratio(seed, off, 1000)
    z2, u2 = O.ratio(seed, off + u1, n - 1000)
    assert np.array_equal(np.concatenate([z1, z2]), z) and u1 + u2 == used
    zs, _ = O.ratio(seed, off, n, mu=-1.0, sigma=2.0)
    assert np.allclose(zs, -1.0 + 2.0 * z, rtol=0, atol=1e-13)
    # each accepted value against the formula written out here
    u = (w[0::2] >> np.uint64(11)).astype(np.float64) * 2.0**-53
    v = (w[1::2] >> np.uint64(11)).astype(np.float64) * 2.0**-53
    x = math.sqrt(8 / math.e) * (v - 0.5) / (1 - u)
    keep = x * x <= -4 * np.log1p(-u)
    assert np.allclose(z, x[keep], rtol=1e-14, atol=1e-15)


def check_ratio_distribution(n: int = 1 << 20):
    z, _ = O.ratio(21, 0, n)
    _dist_checks(z)


def check_stats_routines():
    from scipy import special, stats
    g = np.random.Generator(np.random.PCG64(5))
    x = g.standard_normal(50001) * 1.7 + 0.3
    m = O.moments(x)
    assert abs(m[0] - x.mean()) < 1e-12
    assert abs(m[1] - x.var()) < 1e-12
    assert abs(m[2] - stats.skew(x)) < 1e-10
    assert abs(m[3] - stats.kurtosis(x, fisher=False)) < 1e-10
    for z in (-8.0, -3.0, -0.5, 0.0, 0.7, 2.0, 5.0):
        assert abs(O.normal_cdf(z) - special.ndtr(z)) < 1e-15
    d = O.ks_normal(x, 0.3, 1.7)
    assert abs(d - stats.kstest(x, "norm", args=(0.3, 1.7)).statistic) < 1e-12
    # samples whose empirical CDF lies above and below the model, so that the
    # supremum is attained on each side of the step
    for shift in (-0.2, 0.2):
        xs = x + shift
        d = O.ks_normal(xs, 0.3, 1.7)
        assert abs(d - stats.kstest(xs, "norm", args=(0.3, 1.7)).statistic) < 1e-12
    for a, b in ((1.0, 1.3), (1.3, 1.0)):
        y = g.beta(a, b, 10001)
        assert abs(O.ks_uniform(y) - stats.kstest(y, "uniform").statistic) < 1e-12


ALL_CHECKS = [
    check_splitmix_published, check_stream_definitions, check_b1_hand, check_b1_words_definition,
    check_b1_composition, check_polar_hand, check_polar_lattice, check_polar_composition,
    check_polar_accept_rate, check_polar_s_uniform, check_b1_distribution, check_polar_distribution,
    check_stats_routines, check_p2_poly_bound, check_polar2_hand, check_polar2_lattice, check_polar2_vs_polar,
    check_polar2_distribution, check_b2_hand, check_b2_bound, check_b2_vs_b1, check_b2_stream,
    check_b2_distribution, check_b3_hand, check_b3_stream, check_b3_distribution, check_ratio_hand,
    check_ratio_rate, check_ratio_stream, check_ratio_distribution,
]
