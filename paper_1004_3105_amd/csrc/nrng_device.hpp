// nrng_device.hpp -- device-side building blocks of the normal-deviate
// kernels for gfx950: the counter-based uniform source, the per-pair
// transforms of Box-Muller (Algorithm B1) and the Polar method (Algorithm P)
// [Brent 1993, Section 2], of methods B3 (Section 3) and P2 (Section 4) and
// of Algorithm R (Section 5), output conversion and store helpers, and the
// wavefront primitives of the Polar compaction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nrng_launch.hpp"
#include "nrng_b2_poly.hpp"
#include "nrng_p2_poly.hpp"

namespace nrng {

// ---------------------------------------------------------------------------
// Uniform source.  Counter c = seed + offset + i (mod 2^64); hash
// k = SplitMix64 step of c (Steele, Lea, Flood 2014): add the golden-ratio
// increment, then two xor-shift-multiply rounds and a final xor-shift.
// gfx950 executes the 32-bit multiplies of the 64-bit products at full VALU
// rate, so one full hash is 18 VALU instructions.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t c)
{
    uint64_t z = c + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

// Top 32 bits of the hash of counter c, given z = c + kGamma: the low half
// of the last product and of the final xor-shift are never formed.  Loops
// over consecutive counters keep z itself and step it.
__device__ __forceinline__ uint32_t splitmix64_mix_hi(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    uint32_t h = (uint32_t)(z >> 32);
    return h ^ (h >> 31);
}

__device__ __forceinline__ uint32_t splitmix64_hi(uint64_t c) { return splitmix64_mix_hi(c + kGamma); }

// The full hash of counter c, given z = c + kGamma.
__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Runs of counters whose z = c + kGamma share one high word zh (a tile of
// consecutive counters that does not cross a multiple of 2^32 in z; the
// caller checks this once per tile).  With z = zh 2^32 + zl, the first
// round's high half z1h = zh ^ (zh >> 30) and its contribution z1h * C1lo
// to the high word of the first product depend on zh alone, so they are
// formed once per run (in scalar registers when zh is wave-uniform).  Per
// counter the first round then costs a funnel shift and an xor for the low
// half and one 32 x 32 -> 64-bit multiply-add plus a multiply-add on the
// high word for the product, against a 64-bit shift, two xors and four
// multiply instructions in the general form.  The result is SplitMix64's,
// bit for bit.
struct SmRun {
    uint32_t zh;     // high word of z, common to the run
    uint32_t k1;     // low word of (zh ^ (zh >> 30)) * 0x1CE4E5B9
};

__device__ __forceinline__ SmRun sm_run(uint64_t z_any_in_run)
{
    SmRun r;
    r.zh = (uint32_t)(z_any_in_run >> 32);
    r.k1 = (r.zh ^ (r.zh >> 30)) * 0x1CE4E5B9u;
    return r;
}

// (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 mod 2^64 for z = (r.zh, zl).
__device__ __forceinline__ uint64_t sm_round1(const SmRun &r, uint32_t zl)
{
    const uint32_t z1l = zl ^ __builtin_amdgcn_alignbit(r.zh, zl, 30);
    const uint64_t m = (uint64_t)z1l * 0x1CE4E5B9u;
    const uint32_t ph = (uint32_t)(m >> 32) + z1l * 0xBF58476Du + r.k1;
    return ((uint64_t)ph << 32) | (uint32_t)m;
}

// The rest of the hash from the first product p = (z ^ (z >> 30)) * C1:
// its top 32 bits (as splitmix64_mix_hi) or all of it (as splitmix64_mix).
__device__ __forceinline__ uint32_t sm_hi_of(uint64_t p)
{
    p = (p ^ (p >> 27)) * 0x94D049BB133111EBull;
    const uint32_t h = (uint32_t)(p >> 32);
    return h ^ (h >> 31);
}
__device__ __forceinline__ uint64_t sm_full_of(uint64_t p)
{
    p = (p ^ (p >> 27)) * 0x94D049BB133111EBull;
    return p ^ (p >> 31);
}

// The top word of the second product, before the final xor-shift: the top
// word of the hash is h ^ (h >> 31) (sm_hi_of).
__device__ __forceinline__ uint32_t sm_top_raw_of(uint64_t p)
{
    p = (p ^ (p >> 27)) * 0x94D049BB133111EBull;
    return (uint32_t)(p >> 32);
}

// Top 32 bits of the hash, as splitmix64_mix_hi.
__device__ __forceinline__ uint32_t sm_hi(const SmRun &r, uint32_t zl) { return sm_hi_of(sm_round1(r, zl)); }

// The full hash, as splitmix64_mix.
__device__ __forceinline__ uint64_t sm_full(const SmRun &r, uint32_t zl) { return sm_full_of(sm_round1(r, zl)); }

// True when every z in [zb, zb + span) has the high word of zb (span >= 1).
__device__ __forceinline__ bool sm_run_fits(uint64_t zb, uint64_t span)
{
    return (uint64_t)(uint32_t)zb + (span - 1) <= 0xFFFFFFFFull;
}

// Even-odd pairs of counters.  An even z_e and z_o = z_e + 1 differ in bit 0
// only, so z >> 30 is the same for both and the first round's xor-shift
// gives results that differ in bit 0 only: z_o ^ (z_o >> 30) is one more
// than z_e ^ (z_e >> 30) when bit 0 of the latter (bit 30 of z_e) is clear,
// one less when it is set.  The first product is linear in its operand mod
// 2^64, so its value for z_o is the one for z_e plus or minus C1: one 64-bit
// add in place of the first round.  sm_pair_step gives that C1 or -C1 for
// z_e; it is the same for every even z of a range in which bit 30 does not
// change (sm_pair_fits), which also keeps the range's high word (sm_run).
// The results are SplitMix64's, bit for bit.
__device__ __forceinline__ uint64_t sm_pair_step(uint64_t z_e)
{
    return ((z_e >> 30) & 1) ? 0ull - 0xBF58476D1CE4E5B9ull : 0xBF58476D1CE4E5B9ull;
}

// True when every z in [zb, zb + span) has the bit 30 and the high word of
// zb (no multiple of 2^30 inside; span >= 1).
__device__ __forceinline__ bool sm_pair_fits(uint64_t zb, uint64_t span)
{
    return (uint64_t)((uint32_t)zb & 0x3FFFFFFFu) + (span - 1) <= 0x3FFFFFFFull;
}

// ---------------------------------------------------------------------------
// Output element types.  OutT is the storage type; the arithmetic is FP64 for
// double output (the plain FP64 kernels) and FP32 otherwise.
// ---------------------------------------------------------------------------
struct bf16_t { uint16_t bits; };
struct f16_t { uint16_t bits; };

template <typename OutT> struct out_traits;
template <> struct out_traits<double> { using math = double; static constexpr int bytes = 8; };
template <> struct out_traits<float> { using math = float; static constexpr int bytes = 4; };
template <> struct out_traits<bf16_t> { using math = float; static constexpr int bytes = 2; };
template <> struct out_traits<f16_t> { using math = float; static constexpr int bytes = 2; };

// Round-to-nearest-even float -> bfloat16 (values here are always finite).
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f)
{
    uint32_t b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// Round-to-nearest-even float -> binary16 (hardware conversion; subnormal
// halves are kept).
__device__ __forceinline__ uint16_t f32_to_f16_bits(float f)
{
    // FP16 output is the FP32 value rounded to nearest even: two roundings.
    // The empty asm keeps the compiler from fusing the FMA that produced f
    // with this conversion into one mixed-precision FMA (v_fma_mixlo_f16),
    // which rounds once and differs in rare near-tie cases.
    asm("" : "+v"(f));
    _Float16 h = (_Float16)f;
    return __builtin_bit_cast(uint16_t, h);
}

template <typename OutT> __device__ __forceinline__ uint16_t to_bits16(float f);
template <> __device__ __forceinline__ uint16_t to_bits16<bf16_t>(float f) { return f32_to_bf16_bits(f); }
template <> __device__ __forceinline__ uint16_t to_bits16<f16_t>(float f) { return f32_to_f16_bits(f); }

// Store one element.
template <typename OutT> __device__ __forceinline__ void store1(OutT* p, typename out_traits<OutT>::math v);
template <> __device__ __forceinline__ void store1<double>(double* p, double v) { *p = v; }
template <> __device__ __forceinline__ void store1<float>(float* p, float v) { *p = v; }
template <> __device__ __forceinline__ void store1<bf16_t>(bf16_t* p, float v) { ((uint16_t*)p)[0] = f32_to_bf16_bits(v); }
template <> __device__ __forceinline__ void store1<f16_t>(f16_t* p, float v) { ((uint16_t*)p)[0] = f32_to_f16_bits(v); }

// Store a pair (x, y) at p[0], p[1]; one 2-element store when p is aligned to
// the pair size, otherwise two element stores.
template <typename OutT>
__device__ __forceinline__ void store_pair(OutT* p, typename out_traits<OutT>::math x,
                                           typename out_traits<OutT>::math y)
{
    constexpr int B = out_traits<OutT>::bytes;
    if ((reinterpret_cast<uintptr_t>(p) & (2 * B - 1)) == 0) {
        if constexpr (B == 8) {
            typedef double d2 __attribute__((ext_vector_type(2)));
            *reinterpret_cast<d2*>(p) = d2{x, y};
        } else if constexpr (B == 4) {
            typedef float f2 __attribute__((ext_vector_type(2)));
            *reinterpret_cast<f2*>(p) = f2{x, y};
        } else {
            uint32_t w = (uint32_t)to_bits16<OutT>(x) | ((uint32_t)to_bits16<OutT>(y) << 16);
            *reinterpret_cast<uint32_t*>(p) = w;
        }
    } else {
        store1<OutT>(p, x);
        store1<OutT>(p + 1, y);
    }
}

// Store a pair at a pair-aligned p.
template <typename OutT>
__device__ __forceinline__ void store_pair_aligned(OutT* p, typename out_traits<OutT>::math x,
                                                   typename out_traits<OutT>::math y)
{
    constexpr int B = out_traits<OutT>::bytes;
    if constexpr (B == 8) {
        typedef double d2 __attribute__((ext_vector_type(2)));
        *reinterpret_cast<d2*>(p) = d2{x, y};
    } else if constexpr (B == 4) {
        typedef float f2 __attribute__((ext_vector_type(2)));
        *reinterpret_cast<f2*>(p) = f2{x, y};
    } else {
        *reinterpret_cast<uint32_t*>(p) = (uint32_t)to_bits16<OutT>(x) | ((uint32_t)to_bits16<OutT>(y) << 16);
    }
}

// ---------------------------------------------------------------------------
// Conversions of 64-bit integers to float with relative error below 2^-23
// (the high word is converted and scaled, the low word added by an FMA).
// ---------------------------------------------------------------------------
// One v_cvt_f32_u32.  Written as an instruction because the compiler
// otherwise recognises (float)(uint32_t)(q >> 32) as a 64-bit conversion and
// expands it into a normalising shift sequence.
__device__ __forceinline__ float cvt_f32_u32(uint32_t x)
{
    float r;
    asm("v_cvt_f32_u32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// One v_cvt_f32_i32, for the same reason.
__device__ __forceinline__ float cvt_f32_i32(int32_t x)
{
    float r;
    asm("v_cvt_f32_i32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

__device__ __forceinline__ float u64_to_f32_scaled(uint64_t q, float scale_hi, float scale_lo)
{
    const float hi = cvt_f32_u32((uint32_t)(q >> 32));
    const float lo = (float)(uint32_t)q;
    return __builtin_fmaf(hi, scale_hi, lo * scale_lo);
}

// ---------------------------------------------------------------------------
// Algorithm B1 (Section 2): r = sigma sqrt(-2 ln(1 - u)), x = r sin(2 pi v) + mu,
// y = r cos(2 pi v) + mu, with u = (ku >> 11) 2^-53 and v = (kv >> 11) 2^-53.
// ---------------------------------------------------------------------------

// FP64 evaluation, in the order of the algorithm with no fused operations
// (contraction is switched off in each FP64 evaluation below): 1 - u is
// exact, the angle is the rounded product (2 pi) v.
__device__ __forceinline__ void b1_pair_f64(uint64_t ku, uint64_t kv, double mu, double sigma, double& x,
                                            double& y)
{
    // one rounding per operation, as written (the compiler would otherwise
    // fuse a product and a following sum into an FMA)
#pragma clang fp contract(off)
    double u = (double)(ku >> 11) * 0x1p-53;
    double v = (double)(kv >> 11) * 0x1p-53;
    double r = sigma * sqrt(-2.0 * log(1.0 - u));
    double t = (2.0 * 3.141592653589793115997963) * v;   // 2 fl(pi), exact doubling
    double s, c;
    sincos(t, &s, &c);
    x = r * s + mu;
    y = r * c + mu;
}

// FP32 evaluation.
//  * ln(1 - u) with full relative accuracy for every u: with t = u 2^64 (the
//    53 significant bits of the hash) and q = t for u < 1/2, q = 2^64 - t
//    (= (1 - u) 2^64, exact) otherwise, qf = q 2^-64 rounded once.  For
//    u >= 1/2, ln(1 - u) = ln(qf) directly.  For u < 1/2, y = 1 - qf is
//    rounded; the exact remainder d = (1 - y) - qf (two exact operations)
//    gives ln(1 - u) = ln(y) + ln(1 + d/y) ~= ln(y) + d (2 - y); |d| <= 2^-25,
//    so replacing 1/y by 2 - y (error (1-y)^2/y) costs at most 2^-26 in
//    absolute terms, about 0.2 ulp of |ln(1 - u)| >= 0.69 where it is
//    largest.  One v_log_f32 in all cases.
//  * The angle: v's top 32 bits read as a signed fraction of a turn give
//    v - round(v) in [-1/2, 1/2) exactly; when it exceeds 1/4 in magnitude,
//    half a turn is added (flipping the sign of sin and cos) so the float
//    angle has absolute error at most 2^-27 turns.  v_sin_f32 / v_cos_f32
//    take revolutions.
//  * sigma is folded in as r = sqrt(log2(1 - u) * (-2 ln 2 sigma^2)).
__device__ __forceinline__ float bm_radius_f32(uint64_t ku, float k2)
{
    const uint64_t t = ku & ~0x7FFull;
    const bool lowhalf = t < 0x8000000000000000ull;
    const uint64_t q = lowhalf ? t : (0ull - t);
    const float qf = u64_to_f32_scaled(q, 0x1p-32f, 0x1p-64f);
    const float yv = 1.0f - qf;
    const float d = (1.0f - yv) - qf;
    const float corr = lowhalf ? d * (2.0f - yv) : 0.0f;
    const float arg = lowhalf ? yv : qf;
    const float l2 = __builtin_fmaf(corr, 1.4426950408889634f, __builtin_amdgcn_logf(arg));  // log2(1 - u)
    return __builtin_amdgcn_sqrtf(l2 * k2);
}

__device__ __forceinline__ void b1_pair_f32(uint64_t ku, uint32_t kv_hi, float mu, float k2, float& x,
                                            float& y)
{
    float r = bm_radius_f32(ku, k2);
    // a / 2^32 = v - round(v); flip when a lies outside [-2^30, 2^30)
    const bool flip = (kv_hi + 0x40000000u) >= 0x80000000u;
    const int32_t a = (int32_t)(flip ? (kv_hi ^ 0x80000000u) : kv_hi);
    r = flip ? -r : r;
    const float turns = (float)a * 0x1p-32f;
    const float sn = __builtin_amdgcn_sinf(turns);
    const float cs = __builtin_amdgcn_cosf(turns);
    x = __builtin_fmaf(r, sn, mu);
    y = __builtin_fmaf(r, cs, mu);
}

// ---------------------------------------------------------------------------
// Method B2 (Section 3): B1 with the sine and cosine of the angle 2 pi v - pi
// computed inline: with y = (2 pi v - pi)/16, sin y and cos y from the odd
// and even polynomials of nrng_b2_poly.hpp (t = y^2, nested form), then four
// doublings sin 2y = 2 sin y cos y, cos 2y = 1 - 2 sin^2 y.  Outputs
// r sin(16 y) + mu, then r cos(16 y) + mu.
// ---------------------------------------------------------------------------

// FP64: the order of the method with one rounding per operation, as in
// b1_pair_f64; the radius is B1's.
__device__ __forceinline__ void b2_pair_f64(uint64_t ku, uint64_t kv, double mu, double sigma, double& x,
                                            double& y)
{
#pragma clang fp contract(off)
    const double pi = 3.141592653589793115997963;
    double u = (double)(ku >> 11) * 0x1p-53;
    double v = (double)(kv >> 11) * 0x1p-53;
    double r = sigma * sqrt(-2.0 * log(1.0 - u));
    double yy = ((2.0 * pi) * v - pi) / 16.0;
    double t = yy * yy;
    double s = yy * (kB2SinF64[0] + t * (kB2SinF64[1] + t * (kB2SinF64[2] + t * kB2SinF64[3])));
    double c = kB2CosF64[0] + t * (kB2CosF64[1] + t * (kB2CosF64[2] + t * kB2CosF64[3]));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double s2 = 2.0 * s * c;
        c = 1.0 - 2.0 * s * s;
        s = s2;
    }
    x = r * s + mu;
    y = r * c + mu;
}

// FP32.  The angle 2 pi v - pi is B1's angle minus half a turn, so B2's pair
// is B1's with r negated; B1's reduction to a quarter turn (the signed
// fraction a 2^-32 of a turn, |a| <= 2^30, half a turn added and r negated
// beyond) is reused, so y = 2 pi a 2^-32 / 16 has |y| <= pi/32 and
// 16 y = 2 pi a 2^-32.  Polynomials by FMA; each doubling forms d = 2s
// (exact), s' = d c and c' = 1 - d s with one rounding (FMA).  The absolute
// error of sin 16y and cos 16y is below about 2^-20 (the doublings'
// cancellation in 1 - 2 sin^2 near cos = 0), against about 2^-22 for the
// hardware sine and cosine of B1.
__device__ __forceinline__ void b2_pair_f32(uint64_t ku, uint32_t kv_hi, float mu, float k2, float& x,
                                            float& y)
{
    float r = bm_radius_f32(ku, k2);
    const bool flip = (kv_hi + 0x40000000u) >= 0x80000000u;
    const int32_t a = (int32_t)(flip ? (kv_hi ^ 0x80000000u) : kv_hi);
    r = flip ? r : -r;
    const float yy = cvt_f32_i32(a) * 0x1.921fb6p-34f;          // 2 pi 2^-32 / 16 = pi 2^-35
    const float t = yy * yy;
    float s = yy * __builtin_fmaf(t, __builtin_fmaf(t, __builtin_fmaf(t, kB2SinF32[3], kB2SinF32[2]), kB2SinF32[1]),
                                  kB2SinF32[0]);
    float c = __builtin_fmaf(t, __builtin_fmaf(t, __builtin_fmaf(t, kB2CosF32[3], kB2CosF32[2]), kB2CosF32[1]),
                             kB2CosF32[0]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float d = s + s;
        const float cn = __builtin_fmaf(-d, s, 1.0f);
        s = d * c;
        c = cn;
    }
    x = __builtin_fmaf(r, s, mu);
    y = __builtin_fmaf(r, c, mu);
}

// ---------------------------------------------------------------------------
// Algorithm P (Section 2).  Candidate (X, Y) of signed 32-bit integers,
// x = X 2^-31, y = Y 2^-31, s = S 2^-62 with S = X^2 + Y^2 in uint64.
// Accept iff 0 < S < 2^62 (s < 1 decided exactly; s = 0 rejected).
// ---------------------------------------------------------------------------
// X^2 and Y^2 are at most 2^62, so the sum is exact in uint64 (two signed
// 32 x 32 -> 64-bit multiply-adds).
__device__ __forceinline__ uint64_t polar_S(int32_t X, int32_t Y)
{
    return (uint64_t)((int64_t)X * (int64_t)X) + (uint64_t)((int64_t)Y * (int64_t)Y);
}

// 0 < S < 2^62 as one unsigned comparison of S - 1.
__device__ __forceinline__ bool polar_accept(uint64_t S)
{
    return S - 1 < (1ull << 62) - 1;
}

// The same test from X and Y: S - 1 = X^2 + (Y^2 - 1) by two signed
// 32 x 32 -> 64-bit multiply-adds (the -1 rides in the first one's addend;
// S = 0 gives 2^64 - 1, rejected), then the unsigned comparison.
// Y^2 - 1 as one v_mad_i64_i32 with the addend -1 (written as the
// instruction: the compiler otherwise reassociates (X^2 + (Y^2 - 1)) into
// (X^2 + Y^2) - 1 and spends a 64-bit add on the -1).
__device__ __forceinline__ int64_t sq_minus_one(int32_t y)
{
    int64_t r;
    uint64_t carry;
    asm("v_mad_i64_i32 %0, %1, %2, %2, -1" : "=v"(r), "=s"(carry) : "v"(y));
    return r;
}

__device__ __forceinline__ bool polar_accept_xy(int32_t X, int32_t Y)
{
    const uint64_t sm1 = (uint64_t)((int64_t)X * (int64_t)X + sq_minus_one(Y));
    return sm1 < (1ull << 62) - 1;
}

// Algorithm P's test (P2's with p2 set) decided from the raw top words hx,
// hy of the candidate's two hashes (sm_top_raw_of), without their final
// xor-shift: X = hx ^ (hx >> 31) differs from X' = (int32) hx by at most 1
// (only bit 0 can change), so S' = X'^2 + Y'^2 is within 2^33 of S, and
// S' = 0 exactly when S = 0.  The test on S' therefore equals the test on S
// unless |S' - 2^62| <= 2^34; `band` flags those candidates (about one in
// 10^8), for which the caller decides on X and Y themselves.
template <bool P2>
__device__ __forceinline__ bool polar_screen_raw(uint32_t hx, uint32_t hy, bool &band)
{
    const int32_t x = (int32_t)hx, y = (int32_t)hy;
    const uint64_t sm1 = (uint64_t)((int64_t)x * (int64_t)x + sq_minus_one(y));   // S' - 1
    band = sm1 - ((1ull << 62) - 1 - (1ull << 34)) < (1ull << 35);
    if constexpr (P2)
        return sm1 + 1 < (1ull << 62);      // S' < 2^62 (S' = 0 included)
    else
        return sm1 < (1ull << 62) - 1;      // 0 < S' < 2^62
}

// 2 piece + (bit `lane` of m): one v_addc with the lane mask m as its carry
// in (the compiler otherwise forms the bit by a select and merges it with a
// shift and an or).
__device__ __forceinline__ uint32_t shift_in(uint32_t piece, uint64_t m)
{
    uint32_t r;
    uint64_t carry;
    asm("v_addc_co_u32_e64 %0, %1, %2, %2, %3" : "=v"(r), "=s"(carry) : "v"(piece), "s"(m));
    return r;
}

// FP64 value: s = RNE(S) 2^-62, r = sigma sqrt(-2 ln(s) / s), no fused
// operations.
__device__ __forceinline__ void polar_value_f64(int32_t X, int32_t Y, uint64_t S, double mu, double sigma,
                                                double& zx, double& zy)
{
    // one rounding per operation, as written (the compiler would otherwise
    // fuse a product and a following sum into an FMA)
#pragma clang fp contract(off)
    double s = (double)S * 0x1p-62;
    double r = sigma * sqrt(-2.0 * log(s) / s);
    zx = r * ((double)X * 0x1p-31) + mu;
    zy = r * ((double)Y * 0x1p-31) + mu;
}

// FP32 value.
//  * ln(s): for s <= 1/2, log2 of sf = S 2^-62 rounded once.  For s > 1/2,
//    s = 1 - d with d = (2^62 - S) 2^-62 exact; y = 1 - df rounded (also
//    used as s itself) and the exact remainder e = (1 - y) - df give
//    ln(s) = ln(y) + e (2 - y), as in B1 above.  This keeps ln(s) accurate
//    as s -> 1, where ln(s) cancels.
//  * s < 2^-20 (S < 2^42): ln(s)/s is evaluated in FP64 (exact s; rare).
//  * With l2 = log2(s) (negative for every accepted S), r^2 = -2 ln 2 l2 / s,
//    so sigma r 2^-31 = (l2 kr) / sqrt(-l2 s) with the per-launch constant
//    kr = -sigma sqrt(2 ln 2) 2^-31: one reciprocal square root where
//    r = sqrt(l2 k / s) takes a reciprocal and a square root.  Then
//    z = (sigma r 2^-31) X + mu by an FMA (X as an integer, converted).
// FP32 sigma r 2^-31, r = sqrt(-2 ln(s) / s), for S >= 2^42.
__device__ __forceinline__ float polar_r31_f32(uint64_t S, float kr)
{
    // q = S for s <= 1/2, q = 2^62 - S = d 2^62 (exact) for s > 1/2
    const bool high = S > (1ull << 61);
    const uint64_t q = high ? (1ull << 62) - S : S;
    const float qf = u64_to_f32_scaled(q, 0x1p-30f, 0x1p-62f);
    const float yv = 1.0f - qf;                            // s, rounded, when high
    const float e = (1.0f - yv) - qf;
    const float sf = high ? yv : qf;
    const float corr = high ? e * (2.0f - yv) : 0.0f;
    const float l2 = __builtin_fmaf(corr, 1.4426950408889634f, __builtin_amdgcn_logf(sf));
    return (l2 * kr) * __builtin_amdgcn_rsqf(-(l2 * sf));
}

// The same for S < 2^42 (s < 2^-20), evaluated in FP64 with s exact.
// ln(s) = ln(S) - 62 ln 2; with S = 2^e m, m in [1, 2) (exact), and
// t = (m - 1) / (m + 1) in [0, 1/3), ln(m) = 2 (t + t^3/3 + t^5/5 + ...),
// truncated after t^21 (remainder below 2^-40 relative, far below the FP32
// result's rounding).  The reciprocal and the square root take the hardware
// FP64 approximations plus Newton steps.  A short routine keeps this rare
// path light in registers.
__device__ __forceinline__ double ln_u64_small(uint64_t S)
{
    const int e = 63 - __builtin_clzll(S);                 // S >= 1
    const double m = (double)S * __builtin_ldexp(1.0, -e);  // exact, in [1, 2)
    const double t = (m - 1.0) / (m + 1.0);
    const double t2 = t * t;
    double p = 1.0 / 21;
    p = p * t2 + 1.0 / 19;
    p = p * t2 + 1.0 / 17;
    p = p * t2 + 1.0 / 15;
    p = p * t2 + 1.0 / 13;
    p = p * t2 + 1.0 / 11;
    p = p * t2 + 1.0 / 9;
    p = p * t2 + 1.0 / 7;
    p = p * t2 + 1.0 / 5;
    p = p * t2 + 1.0 / 3;
    p = p * t2 + 1.0;
    return 2.0 * t * p + (double)e * 0.69314718055994530942;
}

// Kept out of line: it runs for about one pair in 10^6, and inlined at its
// two call sites its FP64 temporaries would raise the register count of the
// whole generate kernel (and so lower its occupancy) for every pair.
__device__ __attribute__((noinline)) float polar_r_small(uint64_t S, float sigma)
{
    const double s = (double)S * 0x1p-62;                   // exact
    const double ln_s = ln_u64_small(S) - 62.0 * 0.69314718055994530942;
    const double q = -2.0 * ln_s / s;
    return (float)__builtin_sqrt(q) * sigma;
}

__device__ __forceinline__ bool polar_small(uint64_t S) { return (uint32_t)(S >> 32) < (1u << 10); }   // S < 2^42

__device__ __forceinline__ void polar_value_f32(int32_t X, int32_t Y, uint64_t S, float mu, float kr,
                                                float sigma, float& zx, float& zy)
{
    const float r31 = polar_small(S) ? polar_r_small(S, sigma) * 0x1p-31f : polar_r31_f32(S, kr);
    zx = __builtin_fmaf(r31, (float)X, mu);
    zy = __builtin_fmaf(r31, (float)Y, mu);
}

// a in the lanes whose bit of m is clear, b in the others.  Written as the
// instruction because the compiler otherwise turns a select between two
// costly values into a branch around each, which serialises the pairs a lane
// computes (in a wave of 64 lanes both sides are almost always needed).
// The leading s_nop supplies the wait states that gfx950 requires between a
// transcendental instruction (v_sqrt_f32 and the like) and a VALU
// instruction reading its result: the compiler inserts them for its own
// instructions but not ahead of an inline-assembly reader, which would
// otherwise see the register's previous value.
__device__ __forceinline__ float select_lanes(uint64_t m, float a, float b)
{
    float r;
    asm("s_nop 1\n\tv_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(m));
    return r;
}

// ---------------------------------------------------------------------------
// Method B3 (Section 3).  Per pair three uniforms u1, u2, u3 (counters c,
// c + 1, c + 2): m = max(u1, u2) and u = m^2 (uniform, with sqrt(u) = m);
// r = sigma m h(v), v = (6u - 4)/(4 - 3u), for u <= 8/9, else
// r = sigma sqrt(-ln(1 - u)); t = 2 pi u3 - pi; outputs mu + cos(t) r sqrt(2)
// then mu + sin(t) r sqrt(2).  h is the polynomial of method P2.
// ---------------------------------------------------------------------------

// u > 8/9 with u = RNE_double(m * m), m = mk 2^-53, as the integer test
// mk > kB3SplitM (RNE rounding is monotone, so the set is a ray).  The
// largest mk whose rounded square does not exceed the double 8/9 is found by
// bisection at compile time, with the same double products.
constexpr uint64_t b3_split_m()
{
    uint64_t lo = 0, hi = 1ull << 53;
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        const double m = (double)mid * 0x1p-53;
        if (m * m <= 8.0 / 9.0)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}
constexpr uint64_t kB3SplitM = b3_split_m();

// FP64, in the order of the steps with no fused operations except in the
// polynomial (Horner's rule with FMA).
__device__ __forceinline__ void b3_pair_f64(uint64_t k1, uint64_t k2, uint64_t k3, double mu, double sigma,
                                            double& x, double& y)
{
    // one rounding per operation, as written (the compiler would otherwise
    // fuse a product and a following sum into an FMA)
#pragma clang fp contract(off)
    const double u1 = (double)(k1 >> 11) * 0x1p-53;
    const double u2 = (double)(k2 >> 11) * 0x1p-53;
    const double u3 = (double)(k3 >> 11) * 0x1p-53;
    const double m = u1 > u2 ? u1 : u2;
    const double u = m * m;
    double r;
    if (u > 8.0 / 9.0) {
        r = sigma * sqrt(-log(1.0 - u));
    } else {
        const double v = (6.0 * u - 4.0) / (4.0 - 3.0 * u);
        double h = kP2PolyF64[kP2PolyF64Deg];
#pragma unroll
        for (int k = kP2PolyF64Deg - 1; k >= 0; --k)
            h = __builtin_fma(h, v, kP2PolyF64[k]);
        r = sigma * m * h;
    }
    const double t = (2.0 * 3.141592653589793115997963) * u3 - 3.141592653589793115997963;
    double sn, cs;
    sincos(t, &sn, &cs);
    const double rt = r * 1.4142135623730951;
    x = cs * rt + mu;
    y = sn * rt + mu;
}

// FP32.  ks = sigma sqrt(2), k2 = -2 ln 2 sigma^2.
//  * m from the larger 53-bit integer, rounded once.
//  * u <= 8/9: r sqrt(2) = ks m h(v), v by one reciprocal, h of degree 9.
//  * u > 8/9: 1 - u = (1 - m)(1 + m) with 1 - m = (2^53 - mk) 2^-53 exact
//    before its one rounding, so -ln(1 - u) keeps its relative accuracy;
//    r sqrt(2) = sqrt(log2(1 - u) k2).  Both branches are formed and one is
//    selected.
//  * The angle: u3 - 1/2 is the top word of u3's hash read as a signed
//    fraction of a turn (exact); when it exceeds a quarter turn in magnitude,
//    half a turn is added and r negated, so the float angle has absolute
//    error at most 2^-27 turns.  v_sin_f32 / v_cos_f32 take revolutions.
__device__ __forceinline__ void b3_pair_f32(uint64_t k1, uint64_t k2, uint32_t k3_hi, float mu, float ks, float k2c,
                                            float& x, float& y)
{
    const uint64_t a1 = k1 >> 11, a2 = k2 >> 11;
    const uint64_t mk = a1 > a2 ? a1 : a2;
    const float mf = u64_to_f32_scaled(mk, 0x1p-21f, 0x1p-53f);
    const float uf = mf * mf;
    const float num = __builtin_fmaf(uf, 6.0f, -4.0f);
    const float den = __builtin_fmaf(uf, -3.0f, 4.0f);
    const float v = num * __builtin_amdgcn_rcpf(den);
    float h = kP2PolyF32[kP2PolyF32Deg];
#pragma unroll
    for (int k = kP2PolyF32Deg - 1; k >= 0; --k)
        h = __builtin_fmaf(h, v, kP2PolyF32[k]);
    const float rp = h * mf * ks;
    const float dm = u64_to_f32_scaled((1ull << 53) - mk, 0x1p-21f, 0x1p-53f);   // 1 - m
    const float rl = __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(dm * (1.0f + mf)) * k2c);
    float r = select_lanes(__ballot(mk > kB3SplitM), rp, rl);

    const uint32_t a = k3_hi ^ 0x80000000u;               // (u3 - 1/2) 2^32, as int32
    const bool flip = (a + 0x40000000u) >= 0x80000000u;
    const int32_t af = (int32_t)(flip ? (a ^ 0x80000000u) : a);
    r = flip ? -r : r;
    const float turns = (float)af * 0x1p-32f;
    x = __builtin_fmaf(r, __builtin_amdgcn_cosf(turns), mu);
    y = __builtin_fmaf(r, __builtin_amdgcn_sinf(turns), mu);
}

// ---------------------------------------------------------------------------
// Method P2 (Section 4).  Same candidates as Algorithm P; step 3 rejects only
// s >= 1 (S >= 2^62), so S = 0 is kept (its value is (mu, mu)).  The radius
// factor is sigma sqrt(2) g(s), g(s) = sqrt(-ln(1 - s) / s): for s <= 8/9 a
// polynomial h(v) in v = (6 s - 4) / (4 - 3 s) (Section 3, rho = 1), for
// s > 8/9 the logarithm and square root.  Outputs x r sqrt(2) + mu and
// y r sqrt(2) + mu.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool polar2_accept(uint64_t S) { return S < (1ull << 62); }

// The split s > 8/9, for s = RNE_double(S) 2^-62, as an integer test.
// 8/9 rounded to double, times 2^62, is an integer multiple of 2^9, and
// RNE_double(S) is a multiple of 2^9 for S in [2^61, 2^62), so
// RNE_double(S) <= that value iff S <= it + 256 when the tie at + 256 rounds
// down (to an even multiple), else iff S <= it + 255.
constexpr uint64_t kP2TauS = (uint64_t)((8.0 / 9.0) * 0x1p62);
constexpr uint64_t kP2SplitS = kP2TauS + 256 - ((kP2TauS >> 9) & 1);
__device__ __forceinline__ bool polar2_big(uint64_t S) { return S > kP2SplitS; }

// FP64 value, in the order of the steps with no fused operations except in
// the polynomial (Horner's rule with explicit FMA).
__device__ __forceinline__ void polar2_value_f64(int32_t X, int32_t Y, uint64_t S, double mu, double sigma,
                                                 double& zx, double& zy)
{
    // one rounding per operation, as written (the compiler would otherwise
    // fuse a product and a following sum into an FMA)
#pragma clang fp contract(off)
    const double s = (double)S * 0x1p-62;
    double r;
    if (s > 8.0 / 9.0) {
        r = sigma * sqrt(-log(1.0 - s) / s);
    } else {
        const double v = (6.0 * s - 4.0) / (4.0 - 3.0 * s);
        double h = kP2PolyF64[kP2PolyF64Deg];
#pragma unroll
        for (int k = kP2PolyF64Deg - 1; k >= 0; --k)
            h = __builtin_fma(h, v, kP2PolyF64[k]);
        r = sigma * h;
    }
    const double rt = r * 1.4142135623730951;   // sqrt(2) rounded to double
    zx = rt * ((double)X * 0x1p-31) + mu;
    zy = rt * ((double)Y * 0x1p-31) + mu;
}

// FP32 radius factor times 2^-31: sigma sqrt(2) g(s) 2^-31.  ks31 =
// sigma sqrt(2) 2^-31 and kr = -sigma sqrt(2 ln 2) 2^-31.  Both branches
// are formed in every lane and one is selected.
//  * s <= 8/9: s from the top word of S (absolute error below 2^-30; h has
//    no singularity there, so only absolute accuracy matters), v by one
//    reciprocal, h by Horner's rule with the degree-9 coefficients.
//  * s > 8/9: 1 - s = (2^62 - S) 2^-62 exactly, rounded once, so
//    -ln(1 - s) has full relative accuracy.  With l = log2(1 - s) < 0,
//    sigma sqrt(2) g(s) = sigma sqrt(2 ln 2) sqrt(-l / s), and
//    sigma sqrt(2) g(s) 2^-31 = (l kr) / sqrt(-l s): one reciprocal square
//    root instead of a reciprocal and a square root.
__device__ __forceinline__ float polar2_r31_f32(uint64_t S, float ks31, float kr)
{
    const float hf = cvt_f32_u32((uint32_t)(S >> 32));     // S 2^-32 = s 2^30
    const float num = __builtin_fmaf(hf, 6.0f * 0x1p-30f, -4.0f);
    const float den = __builtin_fmaf(hf, -3.0f * 0x1p-30f, 4.0f);
    const float v = num * __builtin_amdgcn_rcpf(den);
    float h = kP2PolyF32[kP2PolyF32Deg];
#pragma unroll
    for (int k = kP2PolyF32Deg - 1; k >= 0; --k)
        h = __builtin_fmaf(h, v, kP2PolyF32[k]);
    const float tf = u64_to_f32_scaled((1ull << 62) - S, 0x1p-30f, 0x1p-62f);   // 1 - s
    const float sf = hf * 0x1p-30f;
    const float l = __builtin_amdgcn_logf(tf);
    const float rl31 = (l * kr) * __builtin_amdgcn_rsqf(-(l * sf));
    return select_lanes(__ballot(polar2_big(S)), h * ks31, rl31);
}

// ---------------------------------------------------------------------------
// Algorithm R (Section 5; the ratio method in its basic form).  Candidate j
// takes the uniforms u = (k_u >> 11) 2^-53 and v = (k_v >> 11) 2^-53 of
// counters 2j and 2j + 1; x = c (v - 1/2)/(1 - u) with c = sqrt(8/e); the
// candidate is accepted iff x^2 <= -4 ln(1 - u) and then yields sigma x + mu.
// The test is decided in FP64 (the paper's precision), in the oracle's order
// of operations; c is sqrt(8.0 / e) rounded as the host computes it.
// ---------------------------------------------------------------------------
// Kept out of line: the kernels call it only inside the FP32 screen's band
// (ratio_accept_screened) and on the serial continuation path, and inlined
// its FP64 logarithm would raise the register count of the mask and
// generate kernels for every candidate.
__device__ __attribute__((noinline)) bool ratio_accept(uint64_t ku, uint64_t kv, double c)
{
#pragma clang fp contract(off)
    const double u = (double)(ku >> 11) * 0x1p-53;
    const double v = (double)(kv >> 11) * 0x1p-53;
    const double x = c * (v - 0.5) / (1.0 - u);
    return !(x * x > -4.0 * log(1.0 - u));
}

__device__ __forceinline__ double ratio_value_f64(uint64_t ku, uint64_t kv, double c, double mu, double sigma)
{
#pragma clang fp contract(off)
    const double u = (double)(ku >> 11) * 0x1p-53;
    const double v = (double)(kv >> 11) * 0x1p-53;
    const double x = c * (v - 0.5) / (1.0 - u);
    return sigma * x + mu;
}

// FP32 x = c (v - 1/2)/(1 - u) = c dv / du with the 53-bit integers
// dv = (k_v >> 11) - 2^52 and du = 2^53 - (k_u >> 11) >= 1 (the scale 2^-53
// cancels), each converted with relative error below 2^-23; one reciprocal.
// The signed dv is split at bit 21: the low part (below 2^21) converts
// exactly and the high part exactly while |dv| < 2^45, so a small negative dv
// (v just below 1/2, which matters when 1 - u is tiny) is not lost to a
// rounded low word cancelling against the high one.  Also returns du as a
// float (exactly representable scaling by 2^-53 gives 1 - u).
__device__ __forceinline__ float ratio_x_f32(uint64_t ku, uint64_t kv, float c, float& fu)
{
    const int64_t dv = (int64_t)(kv >> 11) - (1ll << 52);
    const uint64_t du = (1ull << 53) - (ku >> 11);
    const float fv = __builtin_fmaf(cvt_f32_i32((int32_t)(dv >> 21)), 0x1p21f,
                                    cvt_f32_u32((uint32_t)dv & 0x1FFFFFu));
    fu = u64_to_f32_scaled(du, 0x1p32f, 1.0f);
    return c * fv * __builtin_amdgcn_rcpf(fu);
}

__device__ __forceinline__ float ratio_value_f32(uint64_t ku, uint64_t kv, float c, float mu, float sigma)
{
    float fu;
    const float x = ratio_x_f32(ku, kv, c, fu);
    return __builtin_fmaf(sigma, x, mu);
}

// The acceptance test of ratio_accept, screened in FP32.  q = x^2 and
// l = -4 ln(1 - u) = -4 ln 2 log2(du 2^-53) are formed in FP32: q has
// relative error below 2^-19 (two conversions, the reciprocal's 1 ulp and
// four roundings), and l absolute error below about 2^-21 (the conversion of
// du moves log2 by at most 1.5 2^-23; v_log_f32 adds about an ulp) plus
// 2^-23 l.  Where |q - l| exceeds 2^-14 (q + l) + 2^-17, at least 16 times
// those bounds, the FP32 comparison is the FP64 one (whose own rounding is
// some 2^-50 relative); inside that band (under 1e-4 of candidates) the
// FP64 test decides.  Same decisions as ratio_accept, without its FP64
// logarithm for nearly every wave.
__device__ __forceinline__ bool ratio_accept_screened(uint64_t ku, uint64_t kv, double c, float c32)
{
    float fu;
    const float x = ratio_x_f32(ku, kv, c32, fu);
    const float q = x * x;
    const float l = -2.7725887222397812f * __builtin_amdgcn_logf(fu * 0x1p-53f);
    bool acc = q <= l;
    if (__builtin_fabsf(q - l) <= __builtin_fmaf(0x1p-14f, q + l, 0x1p-17f))
        acc = ratio_accept(ku, kv, c);
    return acc;
}

// ---------------------------------------------------------------------------
// Wavefront helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Number of set bits of m in lanes below this one.
__device__ __forceinline__ uint32_t rank_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Sixteen dwords at the wave-uniform address p, through the scalar unit
// (p 4-byte aligned, written by an earlier kernel).  The compiler only uses
// scalar loads for memory it can prove unmodified; this one is written out,
// and waits for its data before the block ends.
typedef uint32_t u32x16 __attribute__((ext_vector_type(16)));
__device__ __forceinline__ u32x16 scalar_load16(const void *p)
{
    u32x16 r;
    asm volatile("s_load_dwordx16 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(r) : "s"(p) : "memory");
    return r;
}

// p[i] for a wave-uniform address, through the scalar unit: the constant
// address space tells the compiler that the memory is not written while the
// kernel runs (true of the stream tables, the tile table and the prefixes
// an earlier kernel wrote), so the load goes to an SGPR and what is computed
// from it stays scalar.
template <typename T>
__device__ __forceinline__ T ld_uniform(const T *p, uint64_t i)
{
    return ((const __attribute__((address_space(4))) T *)p)[i];
}

// Lane l's value of v (l wave-uniform).
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l)
{
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Orders one wave's LDS accesses before and after this point for all of its
// lanes: a lane may then read what other lanes of the wave wrote.  The
// fences keep the compiler from moving or forwarding LDS accesses across it
// (a wave's LDS instructions execute in order in hardware).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

}  // namespace nrng
