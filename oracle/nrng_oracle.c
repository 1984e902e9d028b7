/*
 * nrng_oracle.c -- plain, slow, single-threaded FP64 reference for the
 * normal-deviate path: Box-Muller Algorithm B1 and the Polar method,
 * Algorithm P (Section 2), methods B2 and B3 (Section 3), method P2 (Section 4,
 * the Polar method with the radius factor of method B3) and Algorithm R
 * (Section 5, the ratio method in its basic form) of Brent, "Fast Normal Random
 * Number Generators for Vector Processors", 1993.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file.  It is used by the test suite, by the smoke check
 * and by the CPU-baseline leg of the benchmark, and by nothing else.  It
 * shares no code, header, table or constant with the HIP kernels: the
 * uniform generator below is written out again from its published
 * definition.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared (no fused
 * multiply-add, so every line below is one IEEE-754 double operation).
 *
 * Pins (see the tests): the SplitMix64 check sequence, closed-form B1,
 * Polar, P2, B2, B3 and R values for chosen inputs, the paper's error
 * bounds of the P2 polynomial and of B2's sine and cosine against the
 * closed forms, brute-force lattice counts of the Polar acceptance predicate
 * on small grids, the pi/4 and sqrt(pi e)/4 acceptance rates, the
 * uniformity of the accepted s, sample moments and a Kolmogorov-Smirnov
 * statistic against the normal CDF.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

#include "nrng_oracle.h"

/* ------------------------------------------------------------------------
 * Uniform source.  The paper (Section 2) only assumes a generator of
 * uniforms on [0,1) that may return 0 but never 1.  Here the uniforms are a
 * counter-based stream: one SplitMix64 step (Steele, Lea and Flood, OOPSLA
 * 2014) applied to the 64-bit counter  seed + offset + i  (mod 2^64).  A
 * SplitMix64 step adds the golden-ratio increment and then applies the
 * variant-13 mixing function (two xor-shift-multiply rounds and a final
 * xor-shift).
 * --------------------------------------------------------------------- */
uint64_t orc_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* i-th uniform of the stream: the top 53 bits of the hash, scaled by 2^-53,
 * so u lies in [0, 1 - 2^-53] and may be exactly 0 but never 1 (the
 * paper's assumption in Section 2, note a). */
double orc_uniform(uint64_t seed, uint64_t ctr)
{
    return (double)(orc_splitmix64(seed + ctr) >> 11) * 0x1p-53;
}

/* i-th signed 32-bit integer of the stream: the top 32 bits of the hash,
 * read as two's complement.  x = K * 2^-31 is then uniform on [-1, 1), the
 * interval of step 1 of Algorithm P. */
int32_t orc_int32(uint64_t seed, uint64_t ctr)
{
    return (int32_t)(uint32_t)(orc_splitmix64(seed + ctr) >> 32);
}

void orc_hash_block(uint64_t seed, uint64_t offset, uint64_t count, uint64_t *out)
{
    for (uint64_t i = 0; i < count; ++i)
        out[i] = orc_splitmix64(seed + offset + i);
}

void orc_uniform_block(uint64_t seed, uint64_t offset, uint64_t count, double *out)
{
    for (uint64_t i = 0; i < count; ++i)
        out[i] = orc_uniform(seed, offset + i);
}

void orc_int32_block(uint64_t seed, uint64_t offset, uint64_t count, int32_t *out)
{
    for (uint64_t i = 0; i < count; ++i)
        out[i] = orc_int32(seed, offset + i);
}

/* ------------------------------------------------------------------------
 * Algorithm B1 (Box-Muller), Section 2:
 *   r = sigma * sqrt(-2 ln(1 - u));  x = r sin(2 pi v) + mu;  y = r cos(2 pi v) + mu.
 * (1 - u) rather than u because u may be 0 (note a).  The angle is taken
 * literally as 2 pi v with v in [0, 1); note b allows any interval of
 * length 2 pi.  x (the sine) comes first in the output, then y.
 * --------------------------------------------------------------------- */
static void b1_pair(double u, double v, double mu, double sigma, double *x, double *y)
{
    double r = sigma * sqrt(-2.0 * log(1.0 - u));
    double t = (2.0 * M_PI) * v;
    *x = r * sin(t) + mu;
    *y = r * cos(t) + mu;
}

/* B1 from explicit uniforms: pair p uses (u[p], v[p]) and writes out[2p],
 * out[2p+1]. */
void orc_b1_uv(const double *u, const double *v, uint64_t npairs, double mu, double sigma,
               double *out)
{
    for (uint64_t p = 0; p < npairs; ++p)
        b1_pair(u[p], v[p], mu, sigma, &out[2 * p], &out[2 * p + 1]);
}

/* B1 from explicit 64-bit hash words: pair p uses u = (w[2p] >> 11) 2^-53
 * and v = (w[2p+1] >> 11) 2^-53. */
void orc_b1_words(const uint64_t *w, uint64_t npairs, double mu, double sigma, double *out)
{
    for (uint64_t p = 0; p < npairs; ++p) {
        double u = (double)(w[2 * p] >> 11) * 0x1p-53;
        double v = (double)(w[2 * p + 1] >> 11) * 0x1p-53;
        b1_pair(u, v, mu, sigma, &out[2 * p], &out[2 * p + 1]);
    }
}

/* B1 over the counter stream: n normals from uniforms offset, offset+1, ...;
 * pair k uses (u_{2k}, u_{2k+1}).  If n is odd the last pair writes only its
 * first value.  Returns the number of uniforms consumed (2 * ceil(n/2)). */
uint64_t orc_b1(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, double *out)
{
    uint64_t npairs = (n + 1) / 2;
    for (uint64_t k = 0; k < npairs; ++k) {
        double u = orc_uniform(seed, offset + 2 * k);
        double v = orc_uniform(seed, offset + 2 * k + 1);
        double x, y;
        b1_pair(u, v, mu, sigma, &x, &y);
        out[2 * k] = x;
        if (2 * k + 1 < n)
            out[2 * k + 1] = y;
    }
    return 2 * npairs;
}

/* ------------------------------------------------------------------------
 * Algorithm P (the Polar method), Section 2:
 *   1. x, y uniform on [-1, 1);  2. s = x^2 + y^2;  3. reject if s >= 1;
 *   4. r = sigma * sqrt(-2 ln(s) / s), return r x + mu and r y + mu.
 * Here x = X 2^-31 and y = Y 2^-31 for 32-bit signed X, Y, so
 * s = S 2^-62 with the integer S = X^2 + Y^2 (at most 2^63, so it is held in
 * an unsigned 64-bit word).  The test s >= 1 is S >= 2^62, decided exactly
 * in integers.  S = 0 (s = 0) is rejected as well: step 4 would divide by
 * zero, and the paper's suggested substitution of ln(1-s)/(1-s) does not
 * give the same distribution, so the point is simply skipped.  s is S
 * rounded to the nearest double, times 2^-62.
 * --------------------------------------------------------------------- */
int orc_polar_accept(int32_t X, int32_t Y)
{
    uint64_t S = (uint64_t)((int64_t)X * (int64_t)X) + (uint64_t)((int64_t)Y * (int64_t)Y);
    return S != 0 && S < (1ull << 62);
}

static void polar_value(int32_t X, int32_t Y, double mu, double sigma, double *zx, double *zy)
{
    uint64_t S = (uint64_t)((int64_t)X * (int64_t)X) + (uint64_t)((int64_t)Y * (int64_t)Y);
    double s = (double)S * 0x1p-62;
    double r = sigma * sqrt(-2.0 * log(s) / s);
    *zx = r * ((double)X * 0x1p-31) + mu;
    *zy = r * ((double)Y * 0x1p-31) + mu;
}

/* Polar from explicit integer pairs: candidate j is (xy[2j], xy[2j+1]).
 * Accepted candidates are written in increasing j (stable order) as
 * out[2a], out[2a+1] where a counts earlier accepted candidates.  If
 * mask_words is non-null, bit j%64 of mask_words[j/64] is set iff candidate
 * j is accepted.  Returns the number of accepted candidates. */
uint64_t orc_polar_xy(const int32_t *xy, uint64_t ncand, double mu, double sigma, double *out,
                      uint64_t *mask_words)
{
    uint64_t a = 0;
    if (mask_words)
        for (uint64_t w = 0; w < (ncand + 63) / 64; ++w)
            mask_words[w] = 0;
    for (uint64_t j = 0; j < ncand; ++j) {
        int32_t X = xy[2 * j], Y = xy[2 * j + 1];
        if (!orc_polar_accept(X, Y))
            continue;
        if (mask_words)
            mask_words[j / 64] |= 1ull << (j % 64);
        if (out)
            polar_value(X, Y, mu, sigma, &out[2 * a], &out[2 * a + 1]);
        ++a;
    }
    return a;
}

/* Polar over the counter stream: candidate j uses the 32-bit integers at
 * counters offset + 2j and offset + 2j + 1.  Writes exactly n normals (the
 * second value of the last accepted pair is dropped when n is odd) and
 * returns the number of uniforms consumed, 2 (j_last + 1), where j_last is
 * the candidate that supplied the last value (0 when n = 0). */
uint64_t orc_polar(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma,
                   double *out)
{
    uint64_t written = 0, j = 0;
    while (written < n) {
        int32_t X = orc_int32(seed, offset + 2 * j);
        int32_t Y = orc_int32(seed, offset + 2 * j + 1);
        if (orc_polar_accept(X, Y)) {
            double zx, zy;
            polar_value(X, Y, mu, sigma, &zx, &zy);
            out[written++] = zx;
            if (written < n)
                out[written++] = zy;
        }
        ++j;
    }
    return 2 * j;
}

/* Number of accepted candidates among candidates [0, ncand) of the stream
 * starting at counter offset (the predicate only; no values). */
uint64_t orc_polar_count(uint64_t seed, uint64_t offset, uint64_t ncand)
{
    uint64_t a = 0;
    for (uint64_t j = 0; j < ncand; ++j)
        a += (uint64_t)orc_polar_accept(orc_int32(seed, offset + 2 * j),
                                        orc_int32(seed, offset + 2 * j + 1));
    return a;
}

/* Accept masks and output indices for candidates [0, ncand): bit j%64 of
 * mask_words[j/64] is the accept bit of candidate j, and word_prefix[w] is
 * the number of accepted candidates before candidate 64 w (so accepted
 * candidate j lands at output pair word_prefix[j/64] + popcount of the lower
 * bits of its word).  Returns the total accepted. */
uint64_t orc_polar_trace(uint64_t seed, uint64_t offset, uint64_t ncand, uint64_t *mask_words,
                         uint64_t *word_prefix)
{
    uint64_t a = 0;
    for (uint64_t w = 0; w < (ncand + 63) / 64; ++w) {
        uint64_t m = 0;
        if (word_prefix)
            word_prefix[w] = a;
        for (uint64_t b = 0; b < 64 && 64 * w + b < ncand; ++b) {
            uint64_t j = 64 * w + b;
            if (orc_polar_accept(orc_int32(seed, offset + 2 * j),
                                 orc_int32(seed, offset + 2 * j + 1))) {
                m |= 1ull << b;
                ++a;
            }
        }
        mask_words[w] = m;
    }
    return a;
}

/* Values of the accepted candidates in the window [j0, j0 + ncand) of the
 * stream (candidate indices relative to offset), written compactly in stream
 * order; returns how many pairs were written.  Together with
 * orc_polar_count(seed, offset, j0), which gives the output pair index of
 * the first of them, this lets a test check any slice of a long stream. */
uint64_t orc_polar_window(uint64_t seed, uint64_t offset, uint64_t j0, uint64_t ncand, double mu,
                          double sigma, double *out)
{
    uint64_t a = 0;
    for (uint64_t j = j0; j < j0 + ncand; ++j) {
        int32_t X = orc_int32(seed, offset + 2 * j);
        int32_t Y = orc_int32(seed, offset + 2 * j + 1);
        if (orc_polar_accept(X, Y)) {
            polar_value(X, Y, mu, sigma, &out[2 * a], &out[2 * a + 1]);
            ++a;
        }
    }
    return a;
}

/* ------------------------------------------------------------------------
 * Method P2, Section 4 (with the approximation of Section 3).
 *
 * Step 4 of Algorithm P may take -ln of any uniform variable on (0, 1] that
 * is independent of the angle of (x, y) (Knuth's proof), in particular of
 * 1 - s.  The radius factor becomes sigma sqrt(2) g(s) with
 *   g(u) = sqrt(-ln(1 - u) / u),   g(u) = 1 + u/4 + ... near u = 0,
 * the function of method B3.  For s <= 8/9, g(s) = h(v) with
 *   v = (6 s - 4) / (4 - 3 s)  (Section 3, rho = 1: [0, 8/9] -> [-1, 1],
 *   singularities of h at v = +-2),
 * and h is replaced by its Chebyshev series truncated after T_15 (the
 * degree-15 polynomial of Section 3, absolute error below 2e-11 on
 * [-1, 1]).  For s > 8/9 the library ln and sqrt are used.  Outputs are
 * x r sqrt(2) + mu and y r sqrt(2) + mu.
 *
 * Rejection is the literal step 3: s >= 1 only (S >= 2^62).  s = 0 is kept:
 * g(0) = 1 is finite (v = -1), and the pair (0, 0) yields (mu, mu).
 * --------------------------------------------------------------------- */
#define P2_DEGREE 15
#define P2_NODES 64

/* g(u) for 0 <= u < 1 (log1p keeps -ln(1 - u) accurate for small u), in
 * the extended precision of long double: only the coefficients below are
 * computed from it. */
static long double p2_g(long double u)
{
    if (u == 0.0L)
        return 1.0L;
    return sqrtl(-log1pl(-u) / u);
}

/* h(v) = g(u) with u the inverse image of v: u = 4 (v + 1) / (6 + 3 v). */
static long double p2_h_exact(long double v)
{
    return p2_g(4.0L * (v + 1.0L) / (6.0L + 3.0L * v));
}

/* Chebyshev coefficients c[0..degree] of h on [-1, 1], from the discrete
 * orthogonality of T_k at the P2_NODES Chebyshev points t_j = cos(pi (j +
 * 1/2) / N): c_k = (2/N) sum_j h(t_j) T_k(t_j), with c_0 halved.  With 64
 * points the aliased terms are those of degree 113 and above, far below
 * double precision, so these are the coefficients of the series itself.
 * The sums run in long double so that each coefficient is the series'
 * coefficient rounded to double (in double the 64-term sums would leave
 * errors near 1e-15 in each). */
void orc_p2_cheb(int degree, double *c)
{
    long double f[P2_NODES], th[P2_NODES];
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int j = 0; j < P2_NODES; ++j) {
        th[j] = pi * ((long double)j + 0.5L) / (long double)P2_NODES;
        f[j] = p2_h_exact(cosl(th[j]));
    }
    for (int k = 0; k <= degree; ++k) {
        long double sum = 0.0L;
        for (int j = 0; j < P2_NODES; ++j)
            sum += f[j] * cosl((long double)k * th[j]);
        long double ck = 2.0L * sum / (long double)P2_NODES;
        c[k] = (double)(k == 0 ? 0.5L * ck : ck);
    }
}

/* The truncated series sum_{k <= degree} c_k T_k(v), with T_k by the
 * three-term recurrence T_{k+1} = 2 v T_k - T_{k-1}. */
static double cheb_sum(const double *c, int degree, double v)
{
    double t0 = 1.0, t1 = v, sum = c[0];
    if (degree >= 1)
        sum += c[1] * t1;
    for (int k = 2; k <= degree; ++k) {
        double t2 = 2.0 * v * t1 - t0;
        sum += c[k] * t2;
        t0 = t1;
        t1 = t2;
    }
    return sum;
}

/* h(v) by the degree-d truncated series (coefficients recomputed per call:
 * for the pins only). */
double orc_p2_h(int degree, double v)
{
    double c[P2_DEGREE + 8];
    if (degree < 0 || degree > P2_DEGREE + 7)
        return NAN;
    orc_p2_cheb(degree, c);
    return cheb_sum(c, degree, v);
}

int orc_polar2_accept(int32_t X, int32_t Y)
{
    uint64_t S = (uint64_t)((int64_t)X * (int64_t)X) + (uint64_t)((int64_t)Y * (int64_t)Y);
    return S < (1ull << 62);
}

/* Step 4 and 5 of P2 for an accepted (X, Y); c holds the degree-15
 * coefficients. */
static void polar2_value(const double *c, int32_t X, int32_t Y, double mu, double sigma, double *zx,
                         double *zy)
{
    uint64_t S = (uint64_t)((int64_t)X * (int64_t)X) + (uint64_t)((int64_t)Y * (int64_t)Y);
    double s = (double)S * 0x1p-62;
    double r;
    if (s > 8.0 / 9.0) {
        r = sigma * sqrt(-log(1.0 - s) / s);
    } else {
        double v = (6.0 * s - 4.0) / (4.0 - 3.0 * s);
        r = sigma * cheb_sum(c, P2_DEGREE, v);
    }
    double rt = r * M_SQRT2;
    *zx = rt * ((double)X * 0x1p-31) + mu;
    *zy = rt * ((double)Y * 0x1p-31) + mu;
}

/* As orc_polar_xy, for method P2. */
uint64_t orc_polar2_xy(const int32_t *xy, uint64_t ncand, double mu, double sigma, double *out,
                       uint64_t *mask_words)
{
    double c[P2_DEGREE + 1];
    orc_p2_cheb(P2_DEGREE, c);
    uint64_t a = 0;
    if (mask_words)
        for (uint64_t w = 0; w < (ncand + 63) / 64; ++w)
            mask_words[w] = 0;
    for (uint64_t j = 0; j < ncand; ++j) {
        int32_t X = xy[2 * j], Y = xy[2 * j + 1];
        if (!orc_polar2_accept(X, Y))
            continue;
        if (mask_words)
            mask_words[j / 64] |= 1ull << (j % 64);
        if (out)
            polar2_value(c, X, Y, mu, sigma, &out[2 * a], &out[2 * a + 1]);
        ++a;
    }
    return a;
}

/* As orc_polar, for method P2 (same candidates, pairing, order, odd-n rule
 * and consumed count). */
uint64_t orc_polar2(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma,
                    double *out)
{
    double c[P2_DEGREE + 1];
    orc_p2_cheb(P2_DEGREE, c);
    uint64_t written = 0, j = 0;
    while (written < n) {
        int32_t X = orc_int32(seed, offset + 2 * j);
        int32_t Y = orc_int32(seed, offset + 2 * j + 1);
        if (orc_polar2_accept(X, Y)) {
            double zx, zy;
            polar2_value(c, X, Y, mu, sigma, &zx, &zy);
            out[written++] = zx;
            if (written < n)
                out[written++] = zy;
        }
        ++j;
    }
    return 2 * j;
}

uint64_t orc_polar2_count(uint64_t seed, uint64_t offset, uint64_t ncand)
{
    uint64_t a = 0;
    for (uint64_t j = 0; j < ncand; ++j)
        a += (uint64_t)orc_polar2_accept(orc_int32(seed, offset + 2 * j),
                                         orc_int32(seed, offset + 2 * j + 1));
    return a;
}

/* As orc_polar_window, for method P2. */
uint64_t orc_polar2_window(uint64_t seed, uint64_t offset, uint64_t j0, uint64_t ncand, double mu,
                           double sigma, double *out)
{
    double c[P2_DEGREE + 1];
    orc_p2_cheb(P2_DEGREE, c);
    uint64_t a = 0;
    for (uint64_t j = j0; j < j0 + ncand; ++j) {
        int32_t X = orc_int32(seed, offset + 2 * j);
        int32_t Y = orc_int32(seed, offset + 2 * j + 1);
        if (orc_polar2_accept(X, Y)) {
            polar2_value(c, X, Y, mu, sigma, &out[2 * a], &out[2 * a + 1]);
            ++a;
        }
    }
    return a;
}

/* ------------------------------------------------------------------------
 * Method B3, Section 3.  Box-Muller with f(u) = sqrt(-ln(1 - u)) evaluated
 * as sqrt(u) g(u) through the same polynomial h(v) as P2, and the square
 * root avoided by drawing two uniforms: m = max(u1, u2) and u = m^2, which
 * is again uniform on [0, 1) with sqrt(u) = m.  Per pair:
 *   1. u1, u2, u3 uniform;  2. m = max(u1, u2), u = m^2;
 *   3. u > 8/9: r = sigma sqrt(-ln(1 - u)) (library), else
 *      v = (6u - 4)/(4 - 3u) and r = sigma m h(v);
 *   4. s = sin(2 pi u3 - pi), c = cos(2 pi u3 - pi);
 *   5. return mu + c r sqrt(2), then mu + s r sqrt(2).
 * Pair k takes the three consecutive uniforms 3k, 3k + 1, 3k + 2 of the
 * stream, so a stream of n values consumes 3 ceil(n/2) uniforms.
 * --------------------------------------------------------------------- */
static void b3_pair(const double *c, double u1, double u2, double u3, double mu, double sigma, double *x,
                    double *y)
{
    double m = u1 > u2 ? u1 : u2;
    double u = m * m;
    double r;
    if (u > 8.0 / 9.0) {
        r = sigma * sqrt(-log(1.0 - u));
    } else {
        double v = (6.0 * u - 4.0) / (4.0 - 3.0 * u);
        r = sigma * m * cheb_sum(c, P2_DEGREE, v);
    }
    double t = (2.0 * M_PI) * u3 - M_PI;
    double rt = r * M_SQRT2;
    *x = cos(t) * rt + mu;
    *y = sin(t) * rt + mu;
}

/* B3 from explicit uniforms: pair p uses (u1[p], u2[p], u3[p]). */
void orc_b3_u(const double *u1, const double *u2, const double *u3, uint64_t npairs, double mu, double sigma,
              double *out)
{
    double c[P2_DEGREE + 1];
    orc_p2_cheb(P2_DEGREE, c);
    for (uint64_t p = 0; p < npairs; ++p)
        b3_pair(c, u1[p], u2[p], u3[p], mu, sigma, &out[2 * p], &out[2 * p + 1]);
}

/* B3 from explicit 64-bit hash words, three per pair: u_i = (w >> 11) 2^-53. */
void orc_b3_words(const uint64_t *w, uint64_t npairs, double mu, double sigma, double *out)
{
    double c[P2_DEGREE + 1];
    orc_p2_cheb(P2_DEGREE, c);
    for (uint64_t p = 0; p < npairs; ++p) {
        double u1 = (double)(w[3 * p] >> 11) * 0x1p-53;
        double u2 = (double)(w[3 * p + 1] >> 11) * 0x1p-53;
        double u3 = (double)(w[3 * p + 2] >> 11) * 0x1p-53;
        b3_pair(c, u1, u2, u3, mu, sigma, &out[2 * p], &out[2 * p + 1]);
    }
}

/* B3 over the counter stream: n values; returns the uniforms consumed,
 * 3 ceil(n/2). */
uint64_t orc_b3(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, double *out)
{
    double c[P2_DEGREE + 1];
    orc_p2_cheb(P2_DEGREE, c);
    uint64_t npairs = (n + 1) / 2;
    for (uint64_t k = 0; k < npairs; ++k) {
        double u1 = orc_uniform(seed, offset + 3 * k);
        double u2 = orc_uniform(seed, offset + 3 * k + 1);
        double u3 = orc_uniform(seed, offset + 3 * k + 2);
        double x, y;
        b3_pair(c, u1, u2, u3, mu, sigma, &x, &y);
        out[2 * k] = x;
        if (2 * k + 1 < n)
            out[2 * k + 1] = y;
    }
    return 3 * npairs;
}

/* ------------------------------------------------------------------------
 * Method B2, Section 3: Algorithm B1 with the library sine and cosine
 * replaced by an inline approximation.  With the angle 2 pi v - pi and
 * y = (2 pi v - pi)/16, so |y| <= pi/16:
 *   sin y ~= s1 y + s3 y^3 + s5 y^5 + s7 y^7,
 *   cos y ~= c0 + c2 y^2 + c4 y^4 + c6 y^6,
 * and four angle doublings, sin 2y = 2 sin y cos y and
 * cos 2y = 1 - 2 sin^2 y, give sin 16y and cos 16y.  The rest is B1:
 * r = sigma sqrt(-2 ln(1 - u)), outputs r sin(16y) + mu, then
 * r cos(16y) + mu; pair k takes uniforms 2k and 2k + 1.
 *
 * The paper prints neither the coefficients nor their construction, only
 * that the approximations keep the absolute error well below 1e-10.  They
 * are taken here as the Chebyshev series of sin(y)/y and of cos y, as
 * functions of t = y^2 on [0, (pi/16)^2], truncated after T_3 (the
 * construction Section 3 uses for h), and written in powers of t.  The
 * polynomials are evaluated in the nested form y (s1 + t (s3 + t (s5 + t s7)))
 * and c0 + t (c2 + t (c4 + t c6)).
 * --------------------------------------------------------------------- */
#define B2_TAYLOR 14

static long double b2_binom(int n, int k)
{
    long double r = 1.0L;
    for (int i = 1; i <= k; ++i)
        r = r * (long double)(n - k + i) / (long double)i;
    return r;
}

/* The truncated series, computed from the Taylor series f(t) = sum_n f_n t^n
 * term by term (the truncation is linear): with t = (tmax/2)(x + 1) on
 * x in [-1, 1], (x + 1)^n = sum_j C(n, j) x^j and
 * x^j = 2^(1-j) sum_i C(j, i) T_{j-2i}(x) (the T_0 term halved); the terms
 * above T_3 are dropped, the rest is written in powers of x
 * (T_2 = 2x^2 - 1, T_3 = 4x^3 - 3x) and then of t (x = al t - 1,
 * al = 2/tmax).  Each small coefficient is thus a sum of small terms, not
 * the difference of large ones.  Taylor terms past B2_TAYLOR are below
 * 1e-60 on [0, tmax]. */
static void b2_series(const long double *fn, long double tmax, double *m)
{
    const long double al = 2.0L / tmax;
    long double acc[4] = {0.0L, 0.0L, 0.0L, 0.0L};
    long double scale = 1.0L;                       /* (tmax/2)^n */
    for (int n = 0; n < B2_TAYLOR; ++n) {
        long double b[4] = {0.0L, 0.0L, 0.0L, 0.0L};   /* T_0..T_3 part of (x + 1)^n */
        for (int j = 0; j <= n; ++j) {
            for (int i = 0; 2 * i <= j; ++i) {
                int k = j - 2 * i;
                if (k > 3)
                    continue;
                long double w = ldexpl(b2_binom(j, i), 1 - j);
                if (k == 0)
                    w *= 0.5L;
                b[k] += b2_binom(n, j) * w;
            }
        }
        long double p[4] = {b[0] - b[2], b[1] - 3.0L * b[3], 2.0L * b[2], 4.0L * b[3]};
        long double ali = 1.0L;
        for (int i = 0; i < 4; ++i) {
            long double sum = 0.0L;
            for (int j = i; j < 4; ++j)
                sum += p[j] * b2_binom(j, i) * (((j - i) & 1) ? -1.0L : 1.0L);
            acc[i] += fn[n] * scale * ali * sum;
            ali *= al;
        }
        scale *= 0.5L * tmax;
    }
    for (int i = 0; i < 4; ++i)
        m[i] = (double)acc[i];
}

/* s[0..3] = s1, s3, s5, s7 and c[0..3] = c0, c2, c4, c6. */
void orc_b2_coef(double *s, double *c)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double tmax = (pi / 16.0L) * (pi / 16.0L);
    /* sin(y)/y = sum_n (-1)^n t^n / (2n + 1)!,  cos y = sum_n (-1)^n t^n / (2n)! */
    long double fs[B2_TAYLOR], fc[B2_TAYLOR];
    long double fact = 1.0L;                        /* (2n)! */
    for (int n = 0; n < B2_TAYLOR; ++n) {
        if (n > 0)
            fact *= (long double)(2 * n - 1) * (long double)(2 * n);
        long double sg = (n & 1) ? -1.0L : 1.0L;
        fc[n] = sg / fact;
        fs[n] = sg / (fact * (long double)(2 * n + 1));
    }
    b2_series(fs, tmax, s);
    b2_series(fc, tmax, c);
}

/* sin(16y) and cos(16y) from the polynomials at y and four doublings. */
static void b2_sincos16(const double *s, const double *c, double y, double *sn, double *cs)
{
    double t = y * y;
    double sv = y * (s[0] + t * (s[1] + t * (s[2] + t * s[3])));
    double cv = c[0] + t * (c[1] + t * (c[2] + t * c[3]));
    for (int i = 0; i < 4; ++i) {
        double s2 = 2.0 * sv * cv;
        cv = 1.0 - 2.0 * sv * sv;
        sv = s2;
    }
    *sn = sv;
    *cs = cv;
}

/* The approximations to sin(2 pi v - pi) and cos(2 pi v - pi). */
void orc_b2_sincos(double v, double *sn, double *cs)
{
    double s[4], c[4];
    orc_b2_coef(s, c);
    b2_sincos16(s, c, ((2.0 * M_PI) * v - M_PI) / 16.0, sn, cs);
}

static void b2_pair(const double *s, const double *c, double u, double v, double mu, double sigma, double *x,
                    double *y)
{
    double r = sigma * sqrt(-2.0 * log(1.0 - u));
    double sn, cs;
    b2_sincos16(s, c, ((2.0 * M_PI) * v - M_PI) / 16.0, &sn, &cs);
    *x = r * sn + mu;
    *y = r * cs + mu;
}

/* B2 from explicit uniforms: pair p uses (u[p], v[p]). */
void orc_b2_uv(const double *u, const double *v, uint64_t npairs, double mu, double sigma, double *out)
{
    double s[4], c[4];
    orc_b2_coef(s, c);
    for (uint64_t p = 0; p < npairs; ++p)
        b2_pair(s, c, u[p], v[p], mu, sigma, &out[2 * p], &out[2 * p + 1]);
}

/* B2 from explicit 64-bit hash words, two per pair: u = (w >> 11) 2^-53. */
void orc_b2_words(const uint64_t *w, uint64_t npairs, double mu, double sigma, double *out)
{
    double s[4], c[4];
    orc_b2_coef(s, c);
    for (uint64_t p = 0; p < npairs; ++p) {
        double u = (double)(w[2 * p] >> 11) * 0x1p-53;
        double v = (double)(w[2 * p + 1] >> 11) * 0x1p-53;
        b2_pair(s, c, u, v, mu, sigma, &out[2 * p], &out[2 * p + 1]);
    }
}

/* B2 over the counter stream: n values; returns the uniforms consumed,
 * 2 ceil(n/2). */
uint64_t orc_b2(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, double *out)
{
    double s[4], c[4];
    orc_b2_coef(s, c);
    uint64_t npairs = (n + 1) / 2;
    for (uint64_t k = 0; k < npairs; ++k) {
        double u = orc_uniform(seed, offset + 2 * k);
        double v = orc_uniform(seed, offset + 2 * k + 1);
        double x, y;
        b2_pair(s, c, u, v, mu, sigma, &x, &y);
        out[2 * k] = x;
        if (2 * k + 1 < n)
            out[2 * k + 1] = y;
    }
    return 2 * npairs;
}

/* ------------------------------------------------------------------------
 * Algorithm R, Section 5 (the ratio method of Kinderman and Monahan in its
 * basic form): candidate j takes the uniforms u = u_{2j}, v = u_{2j+1};
 *   x = sqrt(8/e) (v - 1/2) / (1 - u);
 *   reject if x^2 > -4 ln(1 - u), else return sigma x + mu.
 * The test is the ratio method's: (1 - u, sqrt(8/e)(v - 1/2)) must lie in
 * the region u' <= exp(-x^2/4) whose area, over the rectangle's, is
 * sqrt(pi e)/4, which gives the 8/sqrt(pi e) = 2.74 uniforms per normal
 * the section states.  (Read literally, the inequality as printed would
 * accept 76% of candidates and return a non-normal variable.)
 * One value per accepted candidate, in increasing j; a stream of n values
 * consumes 2 (j_last + 1) uniforms.  The test is taken in double precision,
 * the precision of the paper's implementations.
 * --------------------------------------------------------------------- */
static double ratio_c(void)
{
    return sqrt(8.0 / M_E);
}

static int ratio_candidate(double c, double u, double v, double *x)
{
    double xv = c * (v - 0.5) / (1.0 - u);
    *x = xv;
    return !(xv * xv > -4.0 * log(1.0 - u));
}

int orc_ratio_accept(double u, double v)
{
    double x;
    return ratio_candidate(ratio_c(), u, v, &x);
}

/* Algorithm R on explicit 64-bit hash words: candidate j is (w[2j], w[2j+1])
 * read as u = (w >> 11) 2^-53, v likewise.  Accepted values are written
 * compactly in order; mask_words as for orc_polar_xy.  Returns the number
 * accepted. */
uint64_t orc_ratio_words(const uint64_t *w, uint64_t ncand, double mu, double sigma, double *out,
                         uint64_t *mask_words)
{
    double c = ratio_c();
    uint64_t a = 0;
    if (mask_words)
        for (uint64_t i = 0; i < (ncand + 63) / 64; ++i)
            mask_words[i] = 0;
    for (uint64_t j = 0; j < ncand; ++j) {
        double u = (double)(w[2 * j] >> 11) * 0x1p-53;
        double v = (double)(w[2 * j + 1] >> 11) * 0x1p-53;
        double x;
        if (!ratio_candidate(c, u, v, &x))
            continue;
        if (mask_words)
            mask_words[j / 64] |= 1ull << (j % 64);
        if (out)
            out[a] = sigma * x + mu;
        ++a;
    }
    return a;
}

/* Algorithm R over the counter stream: n values; returns 2 (j_last + 1). */
uint64_t orc_ratio(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, double *out)
{
    double c = ratio_c();
    uint64_t written = 0, j = 0;
    while (written < n) {
        double u = orc_uniform(seed, offset + 2 * j);
        double v = orc_uniform(seed, offset + 2 * j + 1);
        double x;
        if (ratio_candidate(c, u, v, &x))
            out[written++] = sigma * x + mu;
        ++j;
    }
    return 2 * j;
}

uint64_t orc_ratio_count(uint64_t seed, uint64_t offset, uint64_t ncand)
{
    double c = ratio_c();
    uint64_t a = 0;
    for (uint64_t j = 0; j < ncand; ++j) {
        double x;
        a += (uint64_t)ratio_candidate(c, orc_uniform(seed, offset + 2 * j), orc_uniform(seed, offset + 2 * j + 1),
                                       &x);
    }
    return a;
}

/* Accept masks and per-word exclusive prefixes of candidates [0, ncand), as
 * orc_polar_trace. */
uint64_t orc_ratio_trace(uint64_t seed, uint64_t offset, uint64_t ncand, uint64_t *mask_words,
                         uint64_t *word_prefix)
{
    double c = ratio_c();
    uint64_t a = 0;
    for (uint64_t wd = 0; wd < (ncand + 63) / 64; ++wd) {
        uint64_t m = 0;
        if (word_prefix)
            word_prefix[wd] = a;
        for (uint64_t b = 0; b < 64 && 64 * wd + b < ncand; ++b) {
            uint64_t j = 64 * wd + b;
            double x;
            if (ratio_candidate(c, orc_uniform(seed, offset + 2 * j), orc_uniform(seed, offset + 2 * j + 1), &x)) {
                m |= 1ull << b;
                ++a;
            }
        }
        mask_words[wd] = m;
    }
    return a;
}

/* Values of the accepted candidates in the window [j0, j0 + ncand), as
 * orc_polar_window (one value per candidate). */
uint64_t orc_ratio_window(uint64_t seed, uint64_t offset, uint64_t j0, uint64_t ncand, double mu, double sigma,
                          double *out)
{
    double c = ratio_c();
    uint64_t a = 0;
    for (uint64_t j = j0; j < j0 + ncand; ++j) {
        double x;
        if (ratio_candidate(c, orc_uniform(seed, offset + 2 * j), orc_uniform(seed, offset + 2 * j + 1), &x))
            out[a++] = sigma * x + mu;
    }
    return a;
}

/* ------------------------------------------------------------------------
 * Statistics for the distribution checks (Section 2: the outputs are
 * independent N(mu, sigma^2); in Algorithm P, s is uniform on [0, 1)).
 * --------------------------------------------------------------------- */

/* Pairwise (cascade) summation of f(x_i) for the central moments. */
static double pw_sum_pow(const double *x, uint64_t n, double c, int p)
{
    if (n <= 64) {
        double s = 0.0;
        for (uint64_t i = 0; i < n; ++i) {
            double d = x[i] - c, t = d;
            for (int k = 1; k < p; ++k)
                t = t * d;
            s += (p == 0) ? 1.0 : t;
        }
        return s;
    }
    uint64_t h = n / 2;
    return pw_sum_pow(x, h, c, p) + pw_sum_pow(x + h, n - h, c, p);
}

/* out[0] = mean, out[1] = variance (1/n), out[2] = skewness, out[3] =
 * kurtosis (not excess: 3 for a normal sample). */
void orc_moments(const double *x, uint64_t n, double *out)
{
    double mean = pw_sum_pow(x, n, 0.0, 1) / (double)n;
    double m2 = pw_sum_pow(x, n, mean, 2) / (double)n;
    double m3 = pw_sum_pow(x, n, mean, 3) / (double)n;
    double m4 = pw_sum_pow(x, n, mean, 4) / (double)n;
    out[0] = mean;
    out[1] = m2;
    out[2] = m3 / (m2 * sqrt(m2));
    out[3] = m4 / (m2 * m2);
}

double orc_normal_cdf(double z)
{
    return 0.5 * erfc(-z / M_SQRT2);
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Kolmogorov-Smirnov statistic D = sup |F_n - F| of the sample x (sorted in
 * place) against F = Phi((z - mu) / sigma) when kind = 0, or against the
 * uniform CDF on [0, 1) when kind = 1. */
double orc_ks(double *x, uint64_t n, int kind, double mu, double sigma)
{
    qsort(x, (size_t)n, sizeof(double), cmp_double);
    double d = 0.0;
    for (uint64_t i = 0; i < n; ++i) {
        double f;
        if (kind == 0)
            f = orc_normal_cdf((x[i] - mu) / sigma);
        else
            f = x[i] < 0.0 ? 0.0 : (x[i] > 1.0 ? 1.0 : x[i]);
        double lo = f - (double)i / (double)n;
        double hi = (double)(i + 1) / (double)n - f;
        if (lo > d)
            d = lo;
        if (hi > d)
            d = hi;
    }
    return d;
}
