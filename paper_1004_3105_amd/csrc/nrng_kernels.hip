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
static const Variant kPolarVariants[] = {{256, 4}, {256, 8}, {512, 4}, {128, 8}};
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
// Polar method.  Candidates are processed in tiles of C = WG * U pairs taken
// in ticket order; candidate j of a tile lives in wave j / (64 U), unroll
// slot (j / 64) % U, lane j % 64, so that one ballot per slot is the accept
// mask of 64 consecutive candidates.  Per tile:
//   1. hash, exact integer predicate, ballots; per-wave counts to LDS;
//   2. the tile aggregate is published (inclusive prefix for a stream's first
//      tile);
//   3. the deviates of the accepted candidates are computed in registers
//      (this hides the look-back latency);
//   4. wave 0 looks back over predecessor status words for the exclusive
//      prefix and publishes the inclusive one;
//   5. each accepted candidate stores its pair at output pair index
//      prefix + (rank within the tile), if that index is below ceil(n/2).
// A stream's last budget tile continues serially with further candidates
// if the budget fell short.  The last workgroup to exit resets the control
// block and, for the device-cursor form, advances the cursor.
// ---------------------------------------------------------------------------
template <typename OutT, int WG, int U, int MODE>
__global__ __launch_bounds__(WG) void polar_kernel(PolarArgs a)
{
    using M = typename out_traits<OutT>::math;
    constexpr int NW = WG / 64;
    constexpr uint64_t C = (uint64_t)WG * U;
    __shared__ uint32_t s_cnt[NW];
    __shared__ uint64_t s_excl;
    __shared__ uint32_t s_t;
    __shared__ uint32_t s_wrote, s_last;

    const uint32_t tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
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
    if (tid == 0)
        s_wrote = 0;
    bool wrote = false;

    for (;;) {
        if (tid == 0)
            s_t = __hip_atomic_fetch_add(&ctl->ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint64_t t = s_t;
        if (t >= T)
            break;

        // ---- the job of tile t
        uint64_t ctr0, P, nn, lt, nts, limit;
        OutT *outp;
        uint64_t *st0;
        uint64_t *cons;
        double mu_d, sigma_d;
        if constexpr (MODE == MODE_BATCHED) {
            const uint32_t j = find_stream(a.tile_start, a.nstreams, t);
            const uint64_t ts = a.tile_start[j], te = a.tile_start[j + 1];
            lt = t - ts;
            nts = te - ts;
            nn = a.ns[j];
            P = (nn + 1) / 2;
            ctr0 = a.seeds[j] + a.offsets[j];
            outp = (OutT *)a.out + a.out_off[j];
            mu_d = a.mus[j];
            sigma_d = a.sigmas[j];
            st0 = a.status + ts;
            cons = a.consumed_arr ? a.consumed_arr + j : nullptr;
            limit = ~0ull;
        } else {
            lt = t;
            nts = T;
            ctr0 = a.seed + single_off;
            outp = (OutT *)a.out;
            mu_d = a.mu;
            sigma_d = a.sigma;
            st0 = a.status;
            if constexpr (MODE == MODE_SINGLE) {
                nn = a.n;
                P = (nn + 1) / 2;
                cons = a.consumed;
                limit = ~0ull;
            } else {
                nn = ~0ull;
                P = ~0ull;
                cons = nullptr;
                limit = a.ncand;
            }
        }
        const Coef<M> cf(mu_d, sigma_d);
        uint64_t cand0 = lt * C;
        bool serial = false;
        uint64_t excl = 0;

        for (;;) {
            // ---- 1. candidates, predicate, ballots
            int32_t X[U], Y[U];
            uint64_t S[U], mk[U];
            uint32_t wcnt = 0;
#pragma unroll
            for (int s = 0; s < U; ++s) {
                const uint64_t j = cand0 + (uint64_t)w * 64 * U + (uint64_t)s * 64 + lane;
                bool inb = true;
                if constexpr (MODE == MODE_XY) {
                    inb = j < limit;
                    X[s] = inb ? a.xy[2 * j] : 0;
                    Y[s] = inb ? a.xy[2 * j + 1] : 0;
                } else {
                    if constexpr (MODE == MODE_TRACE)
                        inb = j < limit;
                    X[s] = (int32_t)splitmix64_hi(ctr0 + 2 * j);
                    Y[s] = (int32_t)splitmix64_hi(ctr0 + 2 * j + 1);
                }
                S[s] = polar_S(X[s], Y[s]);
                mk[s] = __ballot(inb && polar_accept(S[s]));
                wcnt += (uint32_t)__builtin_popcountll(mk[s]);
            }
            if (lane == 0)
                s_cnt[w] = wcnt;
            __syncthreads();
            uint32_t tcnt = 0, wpre = 0;
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                const uint32_t c = s_cnt[k];
                wpre += (k < (int)w) ? c : 0u;
                tcnt += c;
            }
            // ---- 2. publish the aggregate (or the inclusive prefix of tile 0)
            if (!serial && tid == 0)
                st_publish(st0 + lt, st_pack(tag, lt == 0 ? ST_INC : ST_AGG, tcnt));

            // ---- 3. values of the accepted candidates
            M zx[U], zy[U];
            if constexpr (MODE != MODE_TRACE) {
#pragma unroll
                for (int s = 0; s < U; ++s) {
                    zx[s] = 0;
                    zy[s] = 0;
                    if ((mk[s] >> lane) & 1ull)
                        polar_value(X[s], Y[s], S[s], cf, zx[s], zy[s]);
                }
            }

            // ---- 4. look-back
            if (!serial) {
                if (w == 0) {
                    const uint64_t e = lt == 0 ? 0 : lookback(st0, (uint32_t)lt, tag);
                    if (lane == 0) {
                        if (lt != 0)
                            st_publish(st0 + lt, st_pack(tag, ST_INC, e + tcnt));
                        s_excl = e;
                    }
                }
                __syncthreads();
                excl = s_excl;
            }

            // ---- 5. stores
            uint64_t run = excl + wpre;
#pragma unroll
            for (int s = 0; s < U; ++s) {
                const uint64_t m = mk[s];
                if constexpr (MODE == MODE_TRACE || MODE == MODE_XY) {
                    const uint64_t widx = (cand0 + (uint64_t)w * 64 * U + (uint64_t)s * 64) >> 6;
                    if (lane == 0 && widx < (a.ncand + 63) / 64) {
                        a.masks[widx] = m;
                        if (a.word_prefix)
                            a.word_prefix[widx] = run;
                    }
                }
                if constexpr (MODE != MODE_TRACE) {
                    if ((m >> lane) & 1ull) {
                        const uint64_t ai = run + rank_below(m);
                        if (ai < P) {
                            OutT *p = outp + 2 * ai;
                            if (2 * ai + 1 < nn)
                                store_pair<OutT>(p, zx[s], zy[s]);
                            else
                                store1<OutT>(p, zx[s]);
                            if constexpr (MODE == MODE_SINGLE || MODE == MODE_BATCHED) {
                                if (ai == P - 1) {
                                    const uint64_t j = cand0 + (uint64_t)w * 64 * U + (uint64_t)s * 64 + lane;
                                    const uint64_t used = 2 * (j + 1);
                                    if (cons)
                                        *cons = used;
                                    if constexpr (MODE == MODE_SINGLE) {
                                        __hip_atomic_store(&ctl->consumed, used, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                                        wrote = true;
                                    }
                                }
                            }
                        }
                    }
                }
                run += (uint64_t)__builtin_popcountll(m);
            }
            const uint64_t incl = excl + tcnt;
            if constexpr (MODE == MODE_XY) {
                if (tid == 0 && lt == nts - 1 && a.count_out)
                    *a.count_out = incl;
            }
            // ---- continuation past the budget (exact, serial, rare)
            const bool more = (MODE == MODE_SINGLE || MODE == MODE_BATCHED) && (lt == nts - 1) && incl < P;
            if (!more)
                break;
            serial = true;
            excl = incl;
            cand0 += C;
            __syncthreads();   // s_cnt is rewritten by the next pass
        }
    }

    // ---- exit: the last workgroup resets the control block
    if (wrote)
        s_wrote = 1;
    __syncthreads();
    if (tid == 0) {
        uint32_t prev;
        if (s_wrote)
            prev = __hip_atomic_fetch_add(&ctl->exited, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        else
            prev = __hip_atomic_fetch_add(&ctl->exited, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const bool wrap = tag + 1 >= kEpochLimit;
        if (wrap) {
            for (uint64_t i = tid; i < a.status_cap; i += WG)
                a.status[i] = 0;
        }
        if (tid == 0) {
            if constexpr (MODE == MODE_SINGLE) {
                if (a.cursor) {
                    const uint64_t used = __hip_atomic_load(&ctl->consumed, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                    *a.cursor = single_off + used;
                }
            }
            __hip_atomic_store(&ctl->consumed, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    uint64_t tloc = 0, run = nbase;
    for (uint32_t j = j0; j < j1; ++j) {
        const uint64_t n = a.ns[j];
        const uint64_t off = a.out_off ? a.out_off[j] : run;
        run = sat_add(run, n);
        const bool valid = n <= a.out_len && off <= a.out_len - n;
        tloc = sat_add(tloc, valid ? tiles_of(n) : 0);
    }
    uint64_t T;
    const uint64_t tbase = block_exclusive_scan(tloc, sh, T);
    const bool ok = (a.method == 0 || T <= a.status_cap) && T < (1ull << 40);
    run = nbase;
    uint64_t tr = tbase;
    for (uint32_t j = j0; j < j1; ++j) {
        const uint64_t n = a.ns[j];
        const uint64_t off = a.out_off ? a.out_off[j] : run;
        run = sat_add(run, n);
        const bool valid = n <= a.out_len && off <= a.out_len - n;
        const uint64_t tl = (ok && valid) ? tiles_of(n) : 0;
        a.tile_start[j] = ok ? tr : 0;
        tr += tl;
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
    if (tid == 0)
        a.tile_start[a.nstreams] = ok ? T : 0;
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
    case 2: return (const void *)polar_kernel<OutT, 512, 4, MODE>;
    case 3: return (const void *)polar_kernel<OutT, 128, 8, MODE>;
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
