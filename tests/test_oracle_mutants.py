"""Mutation tests of the oracle's pins (CPU only).

Each case plants one plausible mistake in a copy of the oracle's C source
(a dropped term, a wrong sign, shift, index or constant, a transposed
operand), builds it with gcc into a temporary directory, and requires that at
least one pin in oracle_pins.py rejects it.  The real oracle is untouched.
"""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle as O
import oracle_pins as P

MUTANTS = {
    "gamma": ("0x9E3779B97F4A7C15ull", "0x9E3779B97F4A7C17ull"),
    "shift30": ("(z >> 30)", "(z >> 31)"),
    "shift27": ("(z >> 27)", "(z >> 28)"),
    "final_shift": ("return z ^ (z >> 31);", "return z ^ (z >> 32);"),
    "mul2": ("0x94D049BB133111EBull", "0x94D049BB133111EAull"),
    "u_bits": ("orc_splitmix64(seed + ctr) >> 11) * 0x1p-53", "orc_splitmix64(seed + ctr) >> 12) * 0x1p-52"),
    "int_hi": ("(orc_splitmix64(seed + ctr) >> 32)", "(orc_splitmix64(seed + ctr) >> 31)"),
    "counter_no_offset": ("out[i] = orc_splitmix64(seed + offset + i);", "out[i] = orc_splitmix64(seed + i);"),
    "b1_u_not_1mu": ("log(1.0 - u)", "log(u + 0x1p-60)"),
    "b1_drop_2": ("sqrt(-2.0 * log(1.0 - u))", "sqrt(-log(1.0 - u))"),
    "b1_pi": ("(2.0 * M_PI) * v", "M_PI * v"),
    "b1_swap_sincos": ("*x = r * sin(t) + mu;\n    *y = r * cos(t) + mu;", "*x = r * cos(t) + mu;\n    *y = r * sin(t) + mu;"),
    "b1_mu_sign": ("*y = r * cos(t) + mu;", "*y = r * cos(t) - mu;"),
    "b1_sigma_dropped": ("double r = sigma * sqrt(-2.0 * log(1.0 - u));", "double r = sqrt(-2.0 * log(1.0 - u));"),
    "b1_pair_order": ("double u = orc_uniform(seed, offset + 2 * k);\n        double v = orc_uniform(seed, offset + 2 * k + 1);",
                      "double v = orc_uniform(seed, offset + 2 * k);\n        double u = orc_uniform(seed, offset + 2 * k + 1);"),
    "b1_words_shift": ("double v = (double)(w[2 * p + 1] >> 11) * 0x1p-53;", "double v = (double)(w[2 * p + 1] >> 12) * 0x1p-52;"),
    "b1_odd_n": ("if (2 * k + 1 < n)\n            out[2 * k + 1] = y;", "out[2 * k + 1] = y;"),
    "polar_boundary": ("S != 0 && S < (1ull << 62)", "S != 0 && S <= (1ull << 62)"),
    "polar_zero": ("S != 0 && S < (1ull << 62)", "S < (1ull << 62)"),
    "polar_drop_div": ("sqrt(-2.0 * log(s) / s)", "sqrt(-2.0 * log(s))"),
    "polar_drop_2": ("sqrt(-2.0 * log(s) / s)", "sqrt(-log(s) / s)"),
    "polar_scale": ("double s = (double)S * 0x1p-62;", "double s = (double)S * 0x1p-63;"),
    "polar_swap_xy": ("*zx = r * ((double)X * 0x1p-31) + mu;\n    *zy = r * ((double)Y * 0x1p-31) + mu;",
                      "*zx = r * ((double)Y * 0x1p-31) + mu;\n    *zy = r * ((double)X * 0x1p-31) + mu;"),
    "polar_x_scale": ("*zx = r * ((double)X * 0x1p-31) + mu;", "*zx = r * ((double)X * 0x1p-32) + mu;"),
    "polar_sigma": ("double r = sigma * sqrt(-2.0 * log(s) / s);", "double r = sqrt(-2.0 * log(s) / s);"),
    "polar_pairing": ("int32_t X = orc_int32(seed, offset + 2 * j);\n        int32_t Y = orc_int32(seed, offset + 2 * j + 1);\n        if (orc_polar_accept(X, Y)) {\n            double zx, zy;",
                      "int32_t X = orc_int32(seed, offset + 2 * j + 1);\n        int32_t Y = orc_int32(seed, offset + 2 * j);\n        if (orc_polar_accept(X, Y)) {\n            double zx, zy;"),
    "polar_consumed": ("    return 2 * j;\n}", "    return 2 * j + 2;\n}"),
    "polar_odd": ("if (written < n)\n                out[written++] = zy;", "out[written++] = zy;"),
    "polar_trace_prefix": ("word_prefix[w] = a;", "word_prefix[w] = a + 1;"),
    "polar_window_start": ("for (uint64_t j = j0; j < j0 + ncand; ++j) {", "for (uint64_t j = j0 + 1; j < j0 + ncand; ++j) {"),
    "p2_degree": ("#define P2_DEGREE 15", "#define P2_DEGREE 14"),
    "p2_nodes": ("#define P2_NODES 64", "#define P2_NODES 12"),
    "p2_map": ("double v = (6.0 * s - 4.0) / (4.0 - 3.0 * s);", "double v = (6.0 * s - 4.0) / (4.0 + 3.0 * s);"),
    "p2_inverse_map": ("p2_g(4.0L * (v + 1.0L) / (6.0L + 3.0L * v))", "p2_g(4.0L * (v + 1.0L) / (6.0L - 3.0L * v))"),
    "p2_g_sign": ("return sqrtl(-log1pl(-u) / u);", "return sqrtl(log1pl(u) / u);"),
    "p2_threshold": ("if (s > 8.0 / 9.0) {", "if (s > 0.97) {"),
    "p2_lib_ln_s": ("r = sigma * sqrt(-log(1.0 - s) / s);", "r = sigma * sqrt(-log(s) / s);"),
    "p2_lib_drop_div": ("r = sigma * sqrt(-log(1.0 - s) / s);", "r = sigma * sqrt(-log(1.0 - s));"),
    "p2_sqrt2": ("double rt = r * M_SQRT2;", "double rt = r;"),
    "p2_swap_xy": ("*zx = rt * ((double)X * 0x1p-31) + mu;\n    *zy = rt * ((double)Y * 0x1p-31) + mu;",
                   "*zx = rt * ((double)Y * 0x1p-31) + mu;\n    *zy = rt * ((double)X * 0x1p-31) + mu;"),
    "p2_accept_zero": ("    return S < (1ull << 62);\n}", "    return S != 0 && S < (1ull << 62);\n}"),
    "p2_cheb_c0": ("c[k] = (double)(k == 0 ? 0.5L * ck : ck);", "c[k] = (double)ck;"),
    "p2_recurrence": ("double t2 = 2.0 * v * t1 - t0;", "double t2 = 2.0 * v * t1 + t0;"),
    "p2_node_phase": ("th[j] = pi * ((long double)j + 0.5L) / (long double)P2_NODES;", "th[j] = pi * (long double)j / (long double)P2_NODES;"),
    "p2_consumed": ("            polar2_value(c, X, Y, mu, sigma, &zx, &zy);\n            out[written++] = zx;\n            if (written < n)\n                out[written++] = zy;\n        }\n        ++j;\n    }\n    return 2 * j;",
                    "            polar2_value(c, X, Y, mu, sigma, &zx, &zy);\n            out[written++] = zx;\n            if (written < n)\n                out[written++] = zy;\n        }\n        ++j;\n    }\n    return 2 * j + 2;"),
    "p2_sigma": ("r = sigma * cheb_sum(c, P2_DEGREE, v);", "r = cheb_sum(c, P2_DEGREE, v);"),
    "b2_taylor": ("#define B2_TAYLOR 14", "#define B2_TAYLOR 4"),
    "b2_three_doublings": ("    for (int i = 0; i < 4; ++i) {\n        double s2", "    for (int i = 0; i < 3; ++i) {\n        double s2"),
    "b2_cos_new_s": ("        cv = 1.0 - 2.0 * sv * sv;\n        sv = s2;", "        sv = s2;\n        cv = 1.0 - 2.0 * sv * sv;"),
    "b2_t_not_squared": ("    double t = y * y;\n    double sv = y *", "    double t = y;\n    double sv = y *"),
    "b2_eighth": ("b2_sincos16(s, c, ((2.0 * M_PI) * v - M_PI) / 16.0, &sn, &cs);", "b2_sincos16(s, c, ((2.0 * M_PI) * v - M_PI) / 8.0, &sn, &cs);"),
    "b2_no_shift": ("b2_sincos16(s, c, ((2.0 * M_PI) * v - M_PI) / 16.0, &sn, &cs);", "b2_sincos16(s, c, ((2.0 * M_PI) * v) / 16.0, &sn, &cs);"),
    "b2_swap": ("    *x = r * sn + mu;\n    *y = r * cs + mu;", "    *x = r * cs + mu;\n    *y = r * sn + mu;"),
    "b2_cheb_t0": ("                if (k == 0)\n                    w *= 0.5L;", "                if (k == 0)\n                    w *= 1.0L;"),
    "b2_binom_sign": ("sum += p[j] * b2_binom(j, i) * (((j - i) & 1) ? -1.0L : 1.0L);", "sum += p[j] * b2_binom(j, i);"),
    "b2_sigma": ("    double r = sigma * sqrt(-2.0 * log(1.0 - u));\n    double sn, cs;", "    double r = sqrt(-2.0 * log(1.0 - u));\n    double sn, cs;"),
    "b2_consumed": ("        b2_pair(s, c, u, v, mu, sigma, &x, &y);\n        out[2 * k] = x;\n        if (2 * k + 1 < n)\n            out[2 * k + 1] = y;\n    }\n    return 2 * npairs;",
                    "        b2_pair(s, c, u, v, mu, sigma, &x, &y);\n        out[2 * k] = x;\n        if (2 * k + 1 < n)\n            out[2 * k + 1] = y;\n    }\n    return 2 * npairs + 2;"),
    "b2_pairing": ("        double u = orc_uniform(seed, offset + 2 * k);\n        double v = orc_uniform(seed, offset + 2 * k + 1);\n        double x, y;\n        b2_pair(",
                   "        double v = orc_uniform(seed, offset + 2 * k);\n        double u = orc_uniform(seed, offset + 2 * k + 1);\n        double x, y;\n        b2_pair("),
    "b3_min": ("double m = u1 > u2 ? u1 : u2;", "double m = u1 < u2 ? u1 : u2;"),
    "b3_u_is_m": ("    double u = m * m;\n    double r;\n    if (u > 8.0 / 9.0) {\n        r = sigma * sqrt(-log(1.0 - u));",
                  "    double u = m;\n    double r;\n    if (u > 8.0 / 9.0) {\n        r = sigma * sqrt(-log(1.0 - u));"),
    "b3_lib_ln_u": ("r = sigma * sqrt(-log(1.0 - u));", "r = sigma * sqrt(-log(u));"),
    "b3_drop_m": ("r = sigma * m * cheb_sum(c, P2_DEGREE, v);", "r = sigma * cheb_sum(c, P2_DEGREE, v);"),
    "b3_angle_shift": ("double t = (2.0 * M_PI) * u3 - M_PI;", "double t = (2.0 * M_PI) * u3;"),
    "b3_swap_cs": ("*x = cos(t) * rt + mu;\n    *y = sin(t) * rt + mu;", "*x = sin(t) * rt + mu;\n    *y = cos(t) * rt + mu;"),
    "b3_sqrt2": ("double rt = r * M_SQRT2;\n    *x = cos(t)", "double rt = r;\n    *x = cos(t)"),
    "b3_threshold": ("    double u = m * m;\n    double r;\n    if (u > 8.0 / 9.0) {", "    double u = m * m;\n    double r;\n    if (u > 0.98) {"),
    "b3_consumed": ("return 3 * npairs;", "return 2 * npairs;"),
    "b3_pairing": ("double u3 = orc_uniform(seed, offset + 3 * k + 2);", "double u3 = orc_uniform(seed, offset + 3 * k + 1);"),
    "b3_words_shift": ("double u3 = (double)(w[3 * p + 2] >> 11) * 0x1p-53;", "double u3 = (double)(w[3 * p + 2] >> 12) * 0x1p-52;"),
    "r_const": ("return sqrt(8.0 / M_E);", "return sqrt(2.0 / M_E);"),
    "r_center": ("double xv = c * (v - 0.5) / (1.0 - u);", "double xv = c * v / (1.0 - u);"),
    "r_u_not_1mu": ("double xv = c * (v - 0.5) / (1.0 - u);", "double xv = c * (v - 0.5) / (u + 0x1p-60);"),
    "r_four": ("return !(xv * xv > -4.0 * log(1.0 - u));", "return !(xv * xv > -2.0 * log(1.0 - u));"),
    "r_direction": ("return !(xv * xv > -4.0 * log(1.0 - u));", "return xv * xv > -4.0 * log(1.0 - u);"),
    "r_printed_form": ("return !(xv * xv > -4.0 * log(1.0 - u));", "return !(-(xv * xv) * log(1.0 - u) > 4.0);"),
    "r_pairing": ("        double u = orc_uniform(seed, offset + 2 * j);\n        double v = orc_uniform(seed, offset + 2 * j + 1);\n        double x;\n        if (ratio_candidate(c, u, v, &x))\n            out[written++]",
                  "        double v = orc_uniform(seed, offset + 2 * j);\n        double u = orc_uniform(seed, offset + 2 * j + 1);\n        double x;\n        if (ratio_candidate(c, u, v, &x))\n            out[written++]"),
    "r_consumed": ("            out[written++] = sigma * x + mu;\n        ++j;\n    }\n    return 2 * j;", "            out[written++] = sigma * x + mu;\n        ++j;\n    }\n    return 2 * j + 2;"),
    "r_sigma": ("            out[written++] = sigma * x + mu;", "            out[written++] = x + mu;"),
    "r_trace_prefix": ("            word_prefix[wd] = a;", "            word_prefix[wd] = a + 1;"),
    "kurtosis": ("out[3] = m4 / (m2 * m2);", "out[3] = m4 / m2;"),
    "skew": ("out[2] = m3 / (m2 * sqrt(m2));", "out[2] = m3 / m2;"),
    "ks_step": ("double hi = (double)(i + 1) / (double)n - f;", "double hi = (double)i / (double)n - f;"),
    "cdf_sign": ("return 0.5 * erfc(-z / M_SQRT2);", "return 0.5 * erfc(z / M_SQRT2);"),
}


@pytest.fixture(scope="module")
def mutant_results():
    """Build every mutant and run the pins on each in its own process, a few
    at a time."""
    from concurrent.futures import ThreadPoolExecutor
    src = O.source_text()
    runner = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mutant_runner.py")
    with tempfile.TemporaryDirectory(prefix="nrng_mut_") as d:
        def one(name):
            old, new = MUTANTS[name]
            if src.count(old) < 1:
                return name, None, "mutation site not found"
            path = O.build_variant(src.replace(old, new, 1), os.path.join(d, "mut_%s.so" % name))
            r = subprocess.run([sys.executable, runner, path], capture_output=True, text=True, timeout=600)
            return name, r.returncode, (r.stdout + r.stderr)[-400:]

        with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            res = {name: (rc, out) for name, rc, out in ex.map(one, sorted(MUTANTS))}
    return res


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, mutant_results):
    rc, out = mutant_results[name]
    assert rc is not None, out
    assert rc != 0, "no pin rejects mutant %s" % name
