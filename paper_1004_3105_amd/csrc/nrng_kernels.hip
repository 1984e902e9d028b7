// nrng_kernels.hip -- HIP kernels for gfx950: Box-Muller (Algorithm B1) and
// the Polar method (Algorithm P) of Brent (1993), Section 2, over single
// streams and over batches of streams, plus the batched tile-table set-up
// kernel and the measurement probes.
#include "nrng_device.hpp"
#include "nrng_launch.hpp"

namespace nrng {

// ---------------------------------------------------------------------------
// Compiled launch variants (workgroup size, per-thread unroll).
// ---------------------------------------------------------------------------
static const Variant kB1Variants[] = {{256, 1}, {256, 2}, {256, 4}, {512, 2}};
// Polar: (workgroup size, candidate slots per lane); a tile is one wave's 64 * unroll candidates
static const Variant kPolarVariants[] = {{256, 4}, {256, 8}, {256, 16}, {512, 8}};
constexpr int kNB1 = sizeof(kB1Variants) / sizeof(kB1Variants[0]);
constexpr int kNPolar = sizeof(kPolarVariants) / sizeof(kPolarVariants[0]);

int b1_variants(const Variant **v) { *v = kB1Variants; return kNB1; }
int polar_variants(const Variant **v) { *v = kPolarVariants; return kNPolar; }

// Per-launch coefficients: FP64 kernels take sigma itself; FP32 kernels take
// -2 ln 2 sigma^2 (r^2 = log2(.) * k2) and sigma.
template <typename M> struct Coef;
template <> struct Coef<double> {
    double mu, k, sigma;
    __device__ Coef(double m, double s) : mu(m), k(s), sigma(s) {}
};
template <> struct Coef<float> {
    float mu, k, sigma;
    __device__ Coef(double m, double s)
        : mu((float)m), k((float)(-1.3862943611198906188 * s * s)), sigma((float)s) {}
};

// One B1 pair from counter c (u from c, v from c + 1).
__device__ __forceinline__ void b1_from_ctr(uint64_t c, const Coef<double> &cf, double &x, double &y)
{
    b1_pair_f64(splitmix64(c), splitmix64(c + 1), cf.mu, cf.k, x, y);
}
__device__ __forceinline__ void b1_from_ctr(uint64_t c, const Coef<float> &cf, float &x, float &y)
{
    b1_pair_f32(splitmix64(c), splitmix64_hi(c + 1), cf.mu, cf.k, x, y);
}
__device__ __forceinline__ void b1_from_words(uint64_t wu, uint64_t wv, const Coef<double> &cf, double &x,
                                              double &y)
{
    b1_pair_f64(wu, wv, cf.mu, cf.k, x, y);
}
__device__ __forceinline__ void b1_from_words(uint64_t wu, uint64_t wv, const Coef<float> &cf, float &x,
                                              float &y)
{
    b1_pair_f32(wu, (uint32_t)(wv >> 32), cf.mu, cf.k, x, y);
}

__device__ __forceinline__ void polar_value(int32_t X, int32_t Y, uint64_t S, const Coef<double> &cf,
                                            double &zx, double &zy)
{
    polar_value_f64(X, Y, S, cf.mu, cf.k, zx, zy);
}
__device__ __forceinline__ void polar_value(int32_t X, int32_t Y, uint64_t S, const Coef<float> &cf, float &zx,
                                            float &zy)
{
    polar_value_f32(X, Y, S, cf.mu, cf.k, cf.sigma, zx, zy);
}

// Split form used by the Polar kernel: the common FP32 path, and the rare
// FP64 path for s < 2^-20, which runs after the main loop so that its
// registers do not count against the main loop's.
__device__ __forceinline__ bool polar_is_rare(uint64_t S, const Coef<double> &) { return false; }
__device__ __forceinline__ bool polar_is_rare(uint64_t S, const Coef<float> &) { return polar_small(S); }

__device__ __forceinline__ void polar_value_common(int32_t X, int32_t Y, uint64_t S, const Coef<double> &cf,
                                                   double &zx, double &zy)
{
    polar_value_f64(X, Y, S, cf.mu, cf.k, zx, zy);
}
__device__ __forceinline__ void polar_value_common(int32_t X, int32_t Y, uint64_t S, const Coef<float> &cf,
                                                   float &zx, float &zy)
{
    const float r = polar_r_f32(S, cf.k);
    zx = __builtin_fmaf(r, (float)X * 0x1p-31f, cf.mu);
    zy = __builtin_fmaf(r, (float)Y * 0x1p-31f, cf.mu);
}

// 16-byte store of 2 * PPL elements (PPL pairs) at a 16-byte aligned p.
template <typename OutT, typename M, int PPL>
__device__ __forceinline__ void store16(OutT *p, const M (&v)[2 * PPL])
{
    if constexpr (sizeof(OutT) == 8) {
        typedef double d2 __attribute__((ext_vector_type(2)));
        *reinterpret_cast<d2 *>(p) = d2{v[0], v[1]};
    } else if constexpr (sizeof(OutT) == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        *reinterpret_cast<f4 *>(p) = f4{v[0], v[1], v[2], v[3]};
    } else {
        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
        u4 w;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            w[i] = (uint32_t)to_bits16<OutT>(v[2 * i]) | ((uint32_t)to_bits16<OutT>(v[2 * i + 1]) << 16);
        *reinterpret_cast<u4 *>(p) = w;
    }
}

// Largest stream index j with ts[j] <= t, for 0 <= t < ts[nstreams]
// (ts non-decreasing, ts[0] = 0).  A 64-ary search: each lane of the wave
// probes one position per round.  Called by all lanes of a wave; the result
// is wave-uniform.
__device__ __forceinline__ uint32_t find_stream(const uint64_t *ts, uint32_t nstreams, uint64_t t)
{
    const uint32_t lane = lane_id();
    uint32_t lo = 0, hi = nstreams;   // ts[lo] <= t < ts[hi]
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + 63) / 64;
        const uint64_t idx = (uint64_t)lo + (uint64_t)step * (lane + 1);
        const bool le = idx < hi && ts[idx] <= t;
        const uint32_t cnt = (uint32_t)__builtin_popcountll(__ballot(le));
        const uint64_t nlo = (uint64_t)lo + (uint64_t)step * cnt;
        const uint64_t nhi = nlo + step;
        lo = (uint32_t)nlo;
        hi = nhi < hi ? (uint32_t)nhi : hi;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// ---------------------------------------------------------------------------
// B1, one stream.  Each lane computes PPL consecutive pairs (16 bytes of
// output) per chunk; a workgroup covers U * WG consecutive chunks per step so
// that every store instruction of a wave writes 1 KiB contiguously.  Grid-
// stride over chunk blocks.
// ---------------------------------------------------------------------------
template <typename OutT, int WG, int U>
__global__ __launch_bounds__(WG) void b1_single_kernel(B1Args a)
{
    using M = typename out_traits<OutT>::math;
    constexpr int PPL = 16 / (2 * out_traits<OutT>::bytes);
    const uint64_t n = a.n, npairs = (n + 1) / 2;
    const uint64_t nchunks = (npairs + PPL - 1) / PPL;
    OutT *out = (OutT *)a.out;
    const bool vec = (reinterpret_cast<uintptr_t>(out) & 15) == 0;
    const Coef<M> cf(a.mu, a.sigma);
    for (uint64_t blk = blockIdx.x; blk * (uint64_t)(U * WG) < nchunks; blk += gridDim.x) {
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint64_t ch = blk * (uint64_t)(U * WG) + (uint64_t)i * WG + threadIdx.x;
            if (ch < nchunks) {
                M v[2 * PPL];
#pragma unroll
                for (int p = 0; p < PPL; ++p)
                    b1_from_ctr(a.ctr0 + 2 * (ch * PPL + p), cf, v[2 * p], v[2 * p + 1]);
                const uint64_t e0 = ch * 2 * PPL;
                if (vec && e0 + 2 * PPL <= n) {
                    store16<OutT, M, PPL>(out + e0, v);
                } else {
#pragma unroll
                    for (int e = 0; e < 2 * PPL; ++e)
                        if (e0 + e < n)
                            store1<OutT>(out + e0 + e, v[e]);
                }
            }
        }
    }
}

// B1 from explicit hash words (test hook): one pair per thread.
template <typename OutT>
__global__ __launch_bounds__(256) void b1_words_kernel(B1Args a, uint64_t npairs)
{
    using M = typename out_traits<OutT>::math;
    const Coef<M> cf(a.mu, a.sigma);
    OutT *out = (OutT *)a.out;
    for (uint64_t p = blockIdx.x * 256ull + threadIdx.x; p < npairs; p += (uint64_t)gridDim.x * 256) {
        M x, y;
        b1_from_words(a.words[2 * p], a.words[2 * p + 1], cf, x, y);
        store1<OutT>(out + 2 * p, x);
        store1<OutT>(out + 2 * p + 1, y);
    }
}

// ---------------------------------------------------------------------------
// B1 over many streams.  Tile t of the table built by prep_kernel belongs to
// stream j = find_stream(t) and covers U * WG * PPL pairs of it.  Streams
// whose output is not 16-byte aligned use pair stores.
// ---------------------------------------------------------------------------
template <typename OutT, int WG, int U>
__global__ __launch_bounds__(WG) void b1_batched_kernel(B1Args a)
{
    using M = typename out_traits<OutT>::math;
    constexpr int PPL = 16 / (2 * out_traits<OutT>::bytes);
    const uint64_t T = a.tile_start[a.nstreams];
    for (uint64_t t = blockIdx.x; t < T; t += gridDim.x) {
        const uint32_t j = find_stream(a.tile_start, a.nstreams, t);
        const uint64_t lt = t - a.tile_start[j];
        const uint64_t n = a.ns[j], npairs = (n + 1) / 2;
        const uint64_t nchunks = (npairs + PPL - 1) / PPL;
        const uint64_t ctr0 = a.seeds[j] + a.offsets[j];
        OutT *out = (OutT *)a.out + a.out_off[j];
        const bool vec = (reinterpret_cast<uintptr_t>(out) & 15) == 0;
        const Coef<M> cf(a.mus[j], a.sigmas[j]);
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint64_t ch = lt * (uint64_t)(U * WG) + (uint64_t)i * WG + threadIdx.x;
            if (ch < nchunks) {
                M v[2 * PPL];
#pragma unroll
                for (int p = 0; p < PPL; ++p)
                    b1_from_ctr(ctr0 + 2 * (ch * PPL + p), cf, v[2 * p], v[2 * p + 1]);
                const uint64_t e0 = ch * 2 * PPL;
                if (vec && e0 + 2 * PPL <= n) {
                    store16<OutT, M, PPL>(out + e0, v);
                } else {
#pragma unroll
                    for (int p = 0; p < PPL; ++p) {
                        const uint64_t e = e0 + 2 * p;
                        if (e + 1 < n)
                            store_pair<OutT>(out + e, v[2 * p], v[2 * p + 1]);
                        else if (e < n)
                            store1<OutT>(out + e, v[2 * p]);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Polar method.  A tile is one wave's work: C = 64 U candidate pairs;
// candidate j of a tile lives in unroll slot j / 64 and lane j % 64, so that
// one ballot per slot is the accept mask of 64 consecutive candidates.  Wave g
// of the grid (W waves in all) takes tiles g, g + W, g + 2W, ...: there is no
// global ticket counter (a single-address atomic would serialise the tiles)
// and no barrier anywhere -- waves only meet through the status words.  Per
// tile:
//   1. hash, exact integer predicate, ballots -> the tile's accepted count;
//   2. the count is published (as the inclusive prefix for a stream's first
//      tile), the wave looks back over predecessor status words for its
//      exclusive prefix and publishes the inclusive one;
//   3. per slot, the accepted lanes compute their deviates and store them at
//      output pair index prefix + (rank within the tile), if below ceil(n/2).
// A stream's last budget tile continues serially with further candidates if
// the budget fell short.  The last wave to exit resets the control block and,
// for the device-cursor form, advances the cursor.
// ---------------------------------------------------------------------------
template <int MODE>
struct PolarSrc {
    uint64_t ctr0;
    const int32_t *xy;
    uint64_t limit;
    __device__ __forceinline__ bool pair(uint64_t j, int32_t &X, int32_t &Y) const
    {
        if constexpr (MODE == MODE_XY) {
            const bool inb = j < limit;
            X = inb ? xy[2 * j] : 0;
            Y = inb ? xy[2 * j + 1] : 0;
            return inb;
        } else {
            X = (int32_t)splitmix64_hi(ctr0 + 2 * j);
            Y = (int32_t)splitmix64_hi(ctr0 + 2 * j + 1);
            return MODE != MODE_TRACE || j < limit;
        }
    }
};

// Accepted count of local tile lt (C candidates), computed by one wave.
template <int MODE>
__device__ uint64_t polar_count_tile(const PolarSrc<MODE> &src, uint64_t lt, uint64_t C)
{
    const uint32_t lane = lane_id();
    uint64_t cnt = 0;
    for (uint64_t b = 0; b < C; b += 64) {
        int32_t X, Y;
        const bool inb = src.pair(lt * C + b + lane, X, Y);
        cnt += (uint64_t)__builtin_popcountll(__ballot(inb && polar_accept(polar_S(X, Y))));
    }
    return cnt;
}

constexpr uint32_t kSpinLimit = 1024;   // polls of a missing status word before computing it

// The per-tile state carried from counting to finishing.
template <typename OutT, int MODE>
struct PolarJob {
    uint64_t t, lt, nts, P, nn, cand0, tcnt;
    OutT *outp;
    uint64_t *st0, *bst, *cons;
    PolarSrc<MODE> src;
    double mu, sigma;
    uint64_t l0;        // block-last tiles: prefix within the block (from counting)
    bool l0_done, l0_inc;
};

template <typename OutT, int WG, int U, int MODE>
__global__ __launch_bounds__(WG) void polar_kernel(PolarArgs a)
{
    using M = typename out_traits<OutT>::math;
    using Job = PolarJob<OutT, MODE>;
    constexpr int NW = WG / 64;
    constexpr uint64_t C = 64ull * U;

    // Each wave parks the candidates of two tiles in its own LDS region: the
    // tile being finished and the next one being counted.  A lane only ever
    // reads back what it wrote itself; the ballots are recomputed from the
    // parked candidates rather than passed between lanes through LDS.
    __shared__ int2 s_xy[NW][2][U][64];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = threadIdx.x >> 6;
    const uint64_t gw = (uint64_t)blockIdx.x * NW + w;
    const uint64_t W = (uint64_t)gridDim.x * NW;
    Ctl *ctl = a.ctl;
    const uint32_t tag = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t single_off = a.offset;
    if constexpr (MODE == MODE_SINGLE) {
        if (a.cursor)
            single_off = *a.cursor;
    }
    uint64_t T;
    if constexpr (MODE == MODE_BATCHED)
        T = a.tile_start[a.nstreams];
    else
        T = a.ntiles;
    bool wrote = false;

    auto make_job = [&](uint64_t t) {
        Job jb;
        jb.t = t;
        jb.src.xy = a.xy;
        jb.src.limit = a.ncand;
        jb.l0 = 0;
        jb.l0_done = jb.l0_inc = false;
        if constexpr (MODE == MODE_BATCHED) {
            const uint32_t j = find_stream(a.tile_start, a.nstreams, t);
            const uint64_t ts = a.tile_start[j], te = a.tile_start[j + 1];
            jb.lt = t - ts;
            jb.nts = te - ts;
            jb.nn = a.ns[j];
            jb.P = (jb.nn + 1) / 2;
            jb.src.ctr0 = a.seeds[j] + a.offsets[j];
            jb.outp = (OutT *)a.out + a.out_off[j];
            jb.mu = a.mus[j];
            jb.sigma = a.sigmas[j];
            jb.st0 = a.status + ts * kStatusStride;
            jb.bst = a.bst + a.block_start[j] * kStatusStride;
            jb.cons = a.consumed_arr ? a.consumed_arr + j : nullptr;
        } else {
            jb.lt = t;
            jb.nts = T;
            jb.src.ctr0 = a.seed + single_off;
            jb.outp = (OutT *)a.out;
            jb.mu = a.mu;
            jb.sigma = a.sigma;
            jb.st0 = a.status;
            jb.bst = a.bst;
            if constexpr (MODE == MODE_SINGLE) {
                jb.nn = a.n;
                jb.P = (jb.nn + 1) / 2;
                jb.cons = a.consumed;
            } else {
                jb.nn = ~0ull;
                jb.P = ~0ull;
                jb.cons = nullptr;
            }
        }
        jb.cand0 = jb.lt * C;
        return jb;
    };

    // 1. hash, exact predicate and ballots of the tile's C candidates,
    // parked in LDS buffer `buf`; returns the accepted count.
    auto count_into = [&](const Job &jb, uint64_t cand0, int buf) {
        uint64_t tcnt = 0;
#pragma unroll
        for (int s = 0; s < U; ++s) {
            const uint64_t j = cand0 + (uint64_t)s * 64 + lane;
            int32_t X, Y;
            const bool inb = jb.src.pair(j, X, Y);
            const uint64_t m = __ballot(inb && polar_accept(polar_S(X, Y)));
            tcnt += (uint64_t)__builtin_popcountll(m);
            s_xy[w][buf][s][lane] = make_int2(X, Y);
        }
        return tcnt;
    };

    // Count a tile and publish its aggregate (inclusive for a stream's first
    // tile).  The last tile of a block also resolves the prefix inside its
    // block and publishes the block aggregate right away, so that later
    // blocks never wait on it.
    auto count = [&](Job &jb, int buf) {
        jb.tcnt = count_into(jb, jb.cand0, buf);
        const uint64_t lt = jb.lt;
        if (lane == 0)
            st_publish(jb.st0 + lt * kStatusStride, st_pack(tag, lt == 0 ? ST_INC : ST_AGG, jb.tcnt));
        const bool block_last = (lt & 63) == 63 || lt + 1 == jb.nts;
        if (block_last && lt != 0) {
            const LookbackRef q{jb.st0, jb.bst, jb.nts};
            const uint32_t k0 = (uint32_t)(lt & 63);
            Resolved r{0, false};
            if (k0)
                r = tiles_window(q, lt, k0, tag, kSpinLimit,
                                 [&](uint64_t t2) { return polar_count_tile<MODE>(jb.src, t2, C); });
            jb.l0 = r.val;
            jb.l0_inc = r.inc;
            jb.l0_done = true;
            if (!r.inc && lane == 0)
                st_publish(jb.bst + (lt >> 6) * kStatusStride, st_pack(tag, ST_AGG, r.val + jb.tcnt));
        }
    };

    // 2.-3. look back, publish the inclusive prefixes, compute and store the
    // deviates of tile jb from LDS buffer buf.
    auto finish = [&](Job &jb, int buf) {
        const uint64_t lt = jb.lt;
        const Coef<M> cf(jb.mu, jb.sigma);
        const bool pair_aligned =
            (reinterpret_cast<uintptr_t>(jb.outp) & (2 * out_traits<OutT>::bytes - 1)) == 0;
        uint64_t excl = 0;
        if (lt != 0) {
            const LookbackRef q{jb.st0, jb.bst, jb.nts};
            auto helper = [&](uint64_t t2) { return polar_count_tile<MODE>(jb.src, t2, C); };
            Resolved r;
            if (jb.l0_done) {
                r = Resolved{jb.l0, jb.l0_inc};
            } else {
                const uint32_t k0 = (uint32_t)(lt & 63);
                r = Resolved{0, false};
                if (k0)
                    r = tiles_window(q, lt, k0, tag, kSpinLimit, helper);
            }
            excl = r.val;
            if (!r.inc)
                excl += lookback_blocks(q, lt >> 6, tag, kSpinLimit, helper);
            if (lane == 0)
                st_publish(jb.st0 + lt * kStatusStride, st_pack(tag, ST_INC, excl + jb.tcnt));
        }
        if (lane == 0 && ((lt & 63) == 63 || lt + 1 == jb.nts))
            st_publish(jb.bst + (lt >> 6) * kStatusStride, st_pack(tag, ST_INC, excl + jb.tcnt));

        const uint64_t P = jb.P, nn = jb.nn;
        auto store = [&](bool all_in, uint64_t ai, M zx, M zy, uint64_t jj) {
            OutT *p = jb.outp + 2 * ai;
            if (all_in) {
                if (pair_aligned)
                    store_pair_aligned<OutT>(p, zx, zy);
                else
                    store_pair<OutT>(p, zx, zy);
            } else if (ai < P) {
                if (2 * ai + 1 < nn)
                    store_pair<OutT>(p, zx, zy);
                else
                    store1<OutT>(p, zx);
                if constexpr (MODE == MODE_SINGLE || MODE == MODE_BATCHED) {
                    if (ai == P - 1) {
                        const uint64_t used = 2 * (jj + 1);
                        if (jb.cons)
                            *jb.cons = used;
                        if constexpr (MODE == MODE_SINGLE) {
                            __hip_atomic_store(&ctl->consumed, used, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            wrote = true;
                        }
                    }
                }
            }
        };

        // the tile itself, from the parked candidates
        {
            const uint64_t cand0 = jb.cand0;
            // fast path: every accepted pair of the tile is needed and complete
            const bool all_in = excl + jb.tcnt <= P && 2 * (excl + jb.tcnt) <= nn;
            uint64_t run = excl;
            uint64_t any_rare = 0;
#pragma unroll
            for (int s = 0; s < U; ++s) {
                const uint64_t jj = cand0 + (uint64_t)s * 64 + lane;
                const int2 xy = s_xy[w][buf][s][lane];
                const uint64_t Ss = polar_S(xy.x, xy.y);
                bool inb = true;
                if constexpr (MODE == MODE_XY || MODE == MODE_TRACE)
                    inb = jj < jb.src.limit;
                const bool acc = inb && polar_accept(Ss);
                const uint64_t m = __ballot(acc);
                if constexpr (MODE == MODE_TRACE || MODE == MODE_XY) {
                    const uint64_t widx = (cand0 + (uint64_t)s * 64) >> 6;
                    if (lane == 0 && widx < (a.ncand + 63) / 64) {
                        a.masks[widx] = m;
                        if (a.word_prefix)
                            a.word_prefix[widx] = run;
                    }
                }
                if constexpr (MODE != MODE_TRACE) {
                    const bool rare = acc && polar_is_rare(Ss, cf);
                    any_rare |= __ballot(rare);
                    if (acc && !rare) {
                        M zx, zy;
                        polar_value_common(xy.x, xy.y, Ss, cf, zx, zy);
                        store(all_in, run + rank_below(m), zx, zy, jj);
                    }
                }
                run += (uint64_t)__builtin_popcountll(m);
            }
            if constexpr (MODE != MODE_TRACE) {
                if (any_rare) {   // wave-uniform; about one tile in 2^14
                    uint64_t run2 = excl;
#pragma unroll 1
                    for (int s = 0; s < U; ++s) {
                        const uint64_t jr = cand0 + (uint64_t)s * 64 + lane;
                        const int2 xy = s_xy[w][buf][s][lane];
                        const uint64_t Sr = polar_S(xy.x, xy.y);
                        bool inb = true;
                        if constexpr (MODE == MODE_XY)
                            inb = jr < jb.src.limit;
                        const uint64_t m = __ballot(inb && polar_accept(Sr));
                        if (((m >> lane) & 1ull) && polar_is_rare(Sr, cf)) {
                            M zx, zy;
                            polar_value(xy.x, xy.y, Sr, cf, zx, zy);
                            store(all_in, run2 + rank_below(m), zx, zy, jr);
                        }
                        run2 += (uint64_t)__builtin_popcountll(m);
                    }
                }
            }
        }
        uint64_t incl = excl + jb.tcnt;
        if constexpr (MODE == MODE_XY) {
            if (lane == 0 && lt == jb.nts - 1 && a.count_out)
                *a.count_out = incl;
        }
        // Continuation past the budget (exact, serial, rare): the stream's
        // last budget tile goes on through further candidates, 64 at a time,
        // with its prefix already known.
        if constexpr (MODE == MODE_SINGLE || MODE == MODE_BATCHED) {
            if (lt == jb.nts - 1) {
                uint64_t j0 = jb.cand0 + C;
#pragma unroll 1
                while (incl < P) {
                    const uint64_t jj = j0 + lane;
                    int32_t X, Y;
                    jb.src.pair(jj, X, Y);
                    const uint64_t Sc = polar_S(X, Y);
                    const bool acc = polar_accept(Sc);
                    const uint64_t m = __ballot(acc);
                    if (acc) {
                        M zx, zy;
                        polar_value(X, Y, Sc, cf, zx, zy);
                        store(false, incl + rank_below(m), zx, zy, jj);
                    }
                    incl += (uint64_t)__builtin_popcountll(m);
                    j0 += 64;
                }
            }
        }
    };

    // software pipeline over this wave's tiles g, g + W, ...: the next tile
    // is counted (and its aggregate published) before the current one looks
    // back, so the predecessors' words are normally visible by then
    if (gw < T) {
        Job cur = make_job(gw);
        count(cur, 0);
        int buf = 0;
        for (;;) {
            const uint64_t tn = cur.t + W;
            const bool has_next = tn < T;
            Job nxt;
            if (has_next) {
                nxt = make_job(tn);
                count(nxt, buf ^ 1);
            }
            finish(cur, buf);
            if (!has_next)
                break;
            cur = nxt;
            buf ^= 1;
        }
    }

    // ---- exit: the last wave resets the control block
    const uint64_t wrote_any = __ballot(wrote);
    if (lane == 0) {
        uint32_t prev;
        if (wrote_any)
            prev = __hip_atomic_fetch_add(&ctl->exited, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        else
            prev = __hip_atomic_fetch_add(&ctl->exited, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wrote = prev == (uint32_t)(W - 1);   // reused: this is the last wave
    }
    const bool last = __ballot(lane == 0 && wrote) != 0;
    if (last) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const bool wrap = tag + 1 >= kEpochLimit;
        if (wrap) {
            for (uint64_t i = lane; i < a.status_cap * kStatusStride; i += 64)
                a.status[i] = 0;
            for (uint64_t i = lane; i < a.bcap * kStatusStride; i += 64)
                a.bst[i] = 0;
        }
        if (lane == 0) {
            if constexpr (MODE == MODE_SINGLE) {
                if (a.cursor) {
                    const uint64_t used = __hip_atomic_load(&ctl->consumed, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                    *a.cursor = single_off + used;
                }
            }
            __hip_atomic_store(&ctl->consumed, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->exited, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->epoch, wrap ? 1u : tag + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// Batched set-up (one workgroup of 1024 threads): per stream, the output
// offset (packed prefix sum when none is given), the range check against
// out_len and the tile count; then the exclusive prefix of the tile counts
// (the tile table) and the initial consumed values.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t sat_add(uint64_t x, uint64_t y)
{
    const uint64_t r = x + y;
    return r < x ? ~0ull : r;
}

__device__ uint64_t block_exclusive_scan(uint64_t v, uint64_t *sh, uint64_t &total)
{
    const uint32_t tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const uint64_t x = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] = sat_add(sh[tid], x);
        __syncthreads();
    }
    const uint64_t incl = sh[tid];
    total = sh[1023];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(1024) void prep_kernel(PrepArgs a)
{
    __shared__ uint64_t sh[1024];
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (a.nstreams + 1023) / 1024;
    const uint64_t j0w = (uint64_t)tid * per;
    const uint32_t j0 = j0w < a.nstreams ? (uint32_t)j0w : a.nstreams;
    const uint32_t j1 = (uint64_t)j0 + per < a.nstreams ? j0 + per : a.nstreams;
    uint64_t total;

    uint64_t nbase = 0;
    if (!a.out_off) {
        uint64_t loc = 0;
        for (uint32_t j = j0; j < j1; ++j)
            loc = sat_add(loc, a.ns[j]);
        nbase = block_exclusive_scan(loc, sh, total);
    }
    auto tiles_of = [&](uint64_t n) -> uint64_t {
        const uint64_t P = (n + 1) / 2;
        if (a.method == 0)
            return (P + a.unit - 1) / a.unit;
        return polar_budget_tiles(P, a.unit);
    };
    uint64_t tloc = 0, bloc = 0, run = nbase;
    for (uint32_t j = j0; j < j1; ++j) {
        const uint64_t n = a.ns[j];
        const uint64_t off = a.out_off ? a.out_off[j] : run;
        run = sat_add(run, n);
        const bool valid = n <= a.out_len && off <= a.out_len - n;
        const uint64_t tl = valid ? tiles_of(n) : 0;
        tloc = sat_add(tloc, tl);
        bloc = sat_add(bloc, (tl + 63) / 64);
    }
    uint64_t T, NB;
    const uint64_t tbase = block_exclusive_scan(tloc, sh, T);
    const uint64_t bbase = block_exclusive_scan(bloc, sh, NB);
    const bool ok = (a.method == 0 || (T <= a.status_cap && NB <= a.block_cap)) && T < (1ull << 40);
    run = nbase;
    uint64_t tr = tbase, br = bbase;
    for (uint32_t j = j0; j < j1; ++j) {
        const uint64_t n = a.ns[j];
        const uint64_t off = a.out_off ? a.out_off[j] : run;
        run = sat_add(run, n);
        const bool valid = n <= a.out_len && off <= a.out_len - n;
        const uint64_t tl = (ok && valid) ? tiles_of(n) : 0;
        a.tile_start[j] = ok ? tr : 0;
        if (a.block_start)
            a.block_start[j] = ok ? br : 0;
        tr += tl;
        br += (tl + 63) / 64;
        if (!a.out_off)
            a.packed_off[j] = valid ? off : 0;
        if (a.consumed) {
            uint64_t c;
            if (!ok || !valid)
                c = ~0ull;
            else if (a.method == 0 || n == 0)
                c = 2 * ((n + 1) / 2);
            else
                c = 0;   // written by the Polar kernel
            a.consumed[j] = c;
        }
    }
    if (tid == 0) {
        a.tile_start[a.nstreams] = ok ? T : 0;
        if (a.block_start)
            a.block_start[a.nstreams] = ok ? NB : 0;
    }
}

// ---------------------------------------------------------------------------
// Probes.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void probe_store_kernel(uint4 *out, uint64_t n16)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n16; i += stride)
        out[i] = make_uint4(0x3F800000u, 0x40000000u, 0x40400000u, (uint32_t)i);
}

__global__ __launch_bounds__(256) void probe_copy_kernel(uint4 *dst, const uint4 *src, uint64_t n16)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

__global__ __launch_bounds__(256) void probe_hash_kernel(uint64_t seed, uint64_t nhash, uint64_t *sink,
                                                         uint64_t sink_len)
{
    const uint64_t g = blockIdx.x * 256ull + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    uint64_t acc = 0;
    for (uint64_t i = g; i < nhash; i += stride)
        acc ^= splitmix64(seed + i);
    if (g < sink_len)
        sink[g] = acc;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <typename OutT>
static const void *b1_single_fn(int vi)
{
    switch (vi) {
    case 0: return (const void *)b1_single_kernel<OutT, 256, 1>;
    case 1: return (const void *)b1_single_kernel<OutT, 256, 2>;
    case 2: return (const void *)b1_single_kernel<OutT, 256, 4>;
    case 3: return (const void *)b1_single_kernel<OutT, 512, 2>;
    }
    return nullptr;
}

template <typename OutT>
static const void *b1_batched_fn(int vi)
{
    switch (vi) {
    case 0: return (const void *)b1_batched_kernel<OutT, 256, 1>;
    case 1: return (const void *)b1_batched_kernel<OutT, 256, 2>;
    case 2: return (const void *)b1_batched_kernel<OutT, 256, 4>;
    case 3: return (const void *)b1_batched_kernel<OutT, 512, 2>;
    }
    return nullptr;
}

template <typename OutT, int MODE>
static const void *polar_fn(int vi)
{
    switch (vi) {
    case 0: return (const void *)polar_kernel<OutT, 256, 4, MODE>;
    case 1: return (const void *)polar_kernel<OutT, 256, 8, MODE>;
    case 2: return (const void *)polar_kernel<OutT, 256, 16, MODE>;
    case 3: return (const void *)polar_kernel<OutT, 512, 8, MODE>;
    }
    return nullptr;
}

template <template <typename> class F>
static const void *by_dtype(int dtype, int vi)
{
    switch (dtype) {
    case 0: return F<double>::get(vi);
    case 1: return F<float>::get(vi);
    case 2: return F<bf16_t>::get(vi);
    case 3: return F<f16_t>::get(vi);
    }
    return nullptr;
}

template <typename OutT> struct B1SingleF { static const void *get(int vi) { return b1_single_fn<OutT>(vi); } };
template <typename OutT> struct B1BatchedF { static const void *get(int vi) { return b1_batched_fn<OutT>(vi); } };
template <typename OutT> struct PolarSingleF { static const void *get(int vi) { return polar_fn<OutT, MODE_SINGLE>(vi); } };
template <typename OutT> struct PolarBatchedF { static const void *get(int vi) { return polar_fn<OutT, MODE_BATCHED>(vi); } };
template <typename OutT> struct PolarXyF { static const void *get(int vi) { return polar_fn<OutT, MODE_XY>(vi); } };
template <typename OutT> struct PolarTraceF { static const void *get(int vi) { return polar_fn<OutT, MODE_TRACE>(vi); } };

static const void *polar_kernel_ptr(int mode, int dtype, int vi)
{
    switch (mode) {
    case MODE_SINGLE: return by_dtype<PolarSingleF>(dtype, vi);
    case MODE_BATCHED: return by_dtype<PolarBatchedF>(dtype, vi);
    case MODE_XY: return by_dtype<PolarXyF>(dtype, vi);
    case MODE_TRACE: return by_dtype<PolarTraceF>(1, vi);
    }
    return nullptr;
}

static int launch_args(const void *fn, uint32_t grid, uint32_t block, void *argp, hipStream_t s)
{
    if (!fn)
        return (int)hipErrorInvalidValue;
    void *args[] = {argp};
    return (int)hipLaunchKernel(fn, dim3(grid), dim3(block), args, 0, s);
}

int launch_b1_single(int dtype, int vi, const B1Args &a, uint32_t grid, hipStream_t s)
{
    B1Args c = a;
    return launch_args(by_dtype<B1SingleF>(dtype, vi), grid, kB1Variants[vi].wg, &c, s);
}

int launch_b1_batched(int dtype, int vi, const B1Args &a, uint32_t grid, hipStream_t s)
{
    B1Args c = a;
    return launch_args(by_dtype<B1BatchedF>(dtype, vi), grid, kB1Variants[vi].wg, &c, s);
}

int launch_b1_words(int dtype, const B1Args &a, uint64_t npairs, hipStream_t s)
{
    B1Args c = a;
    uint64_t np = npairs;
    void *args[] = {&c, &np};
    const void *fn = nullptr;
    switch (dtype) {
    case 0: fn = (const void *)b1_words_kernel<double>; break;
    case 1: fn = (const void *)b1_words_kernel<float>; break;
    case 2: fn = (const void *)b1_words_kernel<bf16_t>; break;
    case 3: fn = (const void *)b1_words_kernel<f16_t>; break;
    default: return (int)hipErrorInvalidValue;
    }
    uint64_t blocks = (npairs + 255) / 256;
    uint32_t grid = (uint32_t)(blocks < 65536 ? (blocks ? blocks : 1) : 65536);
    return (int)hipLaunchKernel(fn, dim3(grid), dim3(256), args, 0, s);
}

int launch_polar(int mode, int dtype, int vi, const PolarArgs &a, uint32_t grid, hipStream_t s)
{
    PolarArgs c = a;
    return launch_args(polar_kernel_ptr(mode, dtype, vi), grid, kPolarVariants[vi].wg, &c, s);
}

int launch_prep(const PrepArgs &a, hipStream_t s)
{
    PrepArgs c = a;
    return launch_args((const void *)prep_kernel, 1, 1024, &c, s);
}

int occupancy_polar(int mode, int dtype, int vi, int *blocks_per_cu)
{
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, polar_kernel_ptr(mode, dtype, vi),
                                                             (int)kPolarVariants[vi].wg, 0);
}

int occupancy_b1(int batched, int dtype, int vi, int *blocks_per_cu)
{
    const void *fn = batched ? by_dtype<B1BatchedF>(dtype, vi) : by_dtype<B1SingleF>(dtype, vi);
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, (int)kB1Variants[vi].wg, 0);
}

int launch_probe_store(void *out, uint64_t nbytes, uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(probe_store_kernel, dim3(grid), dim3(256), 0, s, (uint4 *)out, nbytes / 16);
    return (int)hipGetLastError();
}

int launch_probe_copy(void *dst, const void *src, uint64_t nbytes, uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(probe_copy_kernel, dim3(grid), dim3(256), 0, s, (uint4 *)dst, (const uint4 *)src,
                       nbytes / 16);
    return (int)hipGetLastError();
}

int launch_probe_hash(uint64_t seed, uint64_t nhash, uint64_t *sink, uint64_t sink_len, uint32_t grid,
                      hipStream_t s)
{
    hipLaunchKernelGGL(probe_hash_kernel, dim3(grid), dim3(256), 0, s, seed, nhash, sink, sink_len);
    return (int)hipGetLastError();
}

}  // namespace nrng
