// nrng_kernels_misc.hip -- the non-template kernels (batched set-up, the
// fixed scratch of the allocation-free entry point, probes), the polar scan
// kernel instances, and the launchers that dispatch to the family
// translation units (nrng_kernels_*.hip).
#include <hip/hip_ext.h>

#include "nrng_kernels.hpp"

namespace nrng {

int b1_variants(const Variant **v) { *v = kB1Variants; return kNB1; }
int polar_variants(const Variant **v) { *v = kPolarVariants; return kNPolar; }

// ---------------------------------------------------------------------------
// Batched set-up (one workgroup of 1024 threads): per stream, the output
// offset (packed prefix sum when none is given), the range check against
// out_len and the tile count (Box-Muller family: over n plus the stream's
// line shift, as the batched kernel cuts it); then the exclusive prefix of
// the tile counts (the tile table) and the initial consumed values.
//
// Streams go in chunks of 1024 x kPrepPer; thread t takes kPrepPer
// consecutive streams of a chunk, so its loads are issued together, and the
// two prefixes carry from chunk to chunk.  Each chunk's outputs are written
// as if the table fits; when the total tile count turns out too large for
// the workspace (rare, an error the host reports), or explicit offsets give
// valid streams whose lengths total more than out_len, a second pass over
// the same streams with the same mapping clears the tile table and marks
// every consumed value ~0, so nothing is written.
// ---------------------------------------------------------------------------
constexpr uint32_t kPrepPer = 4;

__global__ __launch_bounds__(1024) void prep_kernel(PrepArgs a)
{
    constexpr uint32_t P = kPrepPer;
    constexpr uint64_t CH = 1024ull * P;
    __shared__ uint64_t sh[32];
    const uint32_t tid = threadIdx.x;
    const uint64_t NS = a.nstreams;
    // B1, B3 and B2 (methods 0, 3 and 5): tiles of `unit` pairs; Polar, P2
    // and R: the candidate budget in words, in tiles of `unit` words
    const bool bm_family = a.method == 0 || a.method == 3 || a.method == 5;
    // tiles of `unit` pairs or words: a shift when unit is a power of two
    // (every launch variant's is), else a 64-bit division
    const bool unit_pow2 = (a.unit & (a.unit - 1)) == 0;
    const uint32_t unit_log2 = (uint32_t)__builtin_ctzll(a.unit);
    auto tiles_in = [&](uint64_t x) -> uint64_t {
        return unit_pow2 ? (x + a.unit - 1) >> unit_log2 : (x + a.unit - 1) / a.unit;
    };

    uint64_t ncarry = 0, tcarry = 0, vcarry = 0;   // saturating sums over earlier chunks
    for (uint64_t base = 0; base < NS; base += CH) {
        const uint64_t j0 = base + (uint64_t)tid * P;
        uint64_t n[P], off[P];
        uint64_t loc = 0;
#pragma unroll
        for (uint32_t i = 0; i < P; ++i) {
            n[i] = j0 + i < NS ? a.ns[j0 + i] : 0;
            off[i] = (a.out_off && j0 + i < NS) ? a.out_off[j0 + i] : 0;
        }
        if (!a.out_off) {
#pragma unroll
            for (uint32_t i = 0; i < P; ++i)
                loc = sat_add(loc, n[i]);
            uint64_t tot;
            uint64_t run = sat_add(ncarry, block_exclusive_scan(loc, sh, tot));
            ncarry = sat_add(ncarry, tot);
#pragma unroll
            for (uint32_t i = 0; i < P; ++i) {
                off[i] = run;
                run = sat_add(run, n[i]);
            }
        }
        bool valid[P];
        uint64_t tl[P], wd[P], tsum = 0, vsum = 0;
#pragma unroll
        for (uint32_t i = 0; i < P; ++i) {
            valid[i] = j0 + i < NS && n[i] <= a.out_len && off[i] <= a.out_len - n[i];
            // the candidate budget of a rejection stream, computed once; a
            // Box-Muller stream's tiles cover its n elements after the line
            // shift
            wd[i] = (!bm_family && valid[i]) ? method_budget_words(a.method, n[i]) : 0;
            const uint64_t sh = a.esize ? line_shift_elems(off[i], a.esize) : 0;
            tl[i] = !valid[i] ? 0 : (bm_family ? (n[i] ? tiles_in((n[i] + sh + 1) / 2) : 0) : tiles_in(wd[i]));
            tsum = sat_add(tsum, tl[i]);
            vsum = sat_add(vsum, valid[i] ? n[i] : 0);
        }
        uint64_t ttot, vtot;
        uint64_t tr = sat_add(tcarry, block_exclusive_scan(tsum, sh, ttot));
        tcarry = sat_add(tcarry, ttot);
        if (a.out_off) {
            // explicit offsets may overlap: the valid streams' total length
            // must still fit out_len (packed streams fit by construction)
            block_exclusive_scan(vsum, sh, vtot);
            vcarry = sat_add(vcarry, vtot);
        }
#pragma unroll
        for (uint32_t i = 0; i < P; ++i) {
            const uint64_t j = j0 + i;
            if (j >= NS)
                break;
            a.tile_start[j] = tr;
            tr += tl[i];
            if (a.stream_words)
                a.stream_words[j] = wd[i];
            if (!a.out_off)
                a.packed_off[j] = valid[i] ? off[i] : 0;
            if (a.consumed) {
                uint64_t c;
                if (!valid[i])
                    c = ~0ull;
                else if (a.method == 3)
                    c = 3 * ((n[i] + 1) / 2);
                else if (a.method == 0 || a.method == 5 || n[i] == 0)
                    c = 2 * ((n[i] + 1) / 2);
                else
                    c = 0;   // written by the Polar generate kernel
                a.consumed[j] = c;
            }
        }
    }
    const uint64_t T = tcarry;
    const bool ok = T < (1ull << 40) && vcarry <= a.out_len &&
                    (bm_family || (T <= a.tile_cap && T * a.unit <= a.word_cap));
    if (!ok) {
        for (uint64_t base = 0; base < NS; base += CH) {
            const uint64_t j0 = base + (uint64_t)tid * P;
#pragma unroll
            for (uint32_t i = 0; i < P; ++i) {
                const uint64_t j = j0 + i;
                if (j >= NS)
                    break;
                a.tile_start[j] = 0;
                if (a.stream_words)
                    a.stream_words[j] = 0;
                if (a.consumed)
                    a.consumed[j] = ~0ull;
            }
        }
    }
    if (tid == 0)
        a.tile_start[NS] = ok ? T : 0;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free Polar entry point: a fixed array in device
// memory (one copy per device, held until the process ends) that stands in
// for the library's growable workspace -- accept masks, tile and chunk
// prefixes and the cursor latch of one single-stream call.  In host code
// the array's name is not a device address; the address is taken once per
// device with hipGetSymbolAddress (that device current) and passed to the
// kernels like any workspace pointer.
// ---------------------------------------------------------------------------
constexpr int kScratchDevs = 64;
static __device__ __align__(256) uint64_t scratch[kScratchBytes / sizeof(uint64_t)];
static void *g_scratch_addr[kScratchDevs];

int scratch_address(int dev, void **addr)
{
    if (dev < 0 || dev >= kScratchDevs)
        return (int)hipErrorInvalidDevice;
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return (int)e;
        g_scratch_addr[dev] = p;
    }
    *addr = g_scratch_addr[dev];
    return (int)hipSuccess;
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

// The store-only ceiling in a chosen form: UNR 16-byte stores per thread
// per step, each thread's stores 256 x 16 bytes apart (so that every store
// instruction of a wave writes 1 KiB contiguously), plain or nontemporal.
template <bool NT, int UNR>
__global__ __launch_bounds__(256) void probe_store_var_kernel(uint4 *out, uint64_t n16)
{
    const uint64_t step = (uint64_t)gridDim.x * 256 * UNR;
    for (uint64_t base = blockIdx.x * 256ull * UNR + threadIdx.x; base < n16; base += step) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const uint64_t i = base + (uint64_t)u * 256;
            if (i < n16) {
                typedef uint32_t u4 __attribute__((ext_vector_type(4)));
                const u4 v = {0x3F800000u, 0x40000000u, 0x40400000u, (uint32_t)i};
                u4 *q = reinterpret_cast<u4 *>(out + i);
                if constexpr (NT)
                    __builtin_nontemporal_store(v, q);
                else
                    *q = v;
            }
        }
    }
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
static bool b1_vi_ok(int vi) { return vi >= 0 && vi < kNB1; }

// The Box-Muller-family kernel of (batched, method, dtype, variant).
static const void *b1_ptr(int batched, int bm, int dtype, int vi)
{
    if (!b1_vi_ok(vi))
        return nullptr;
    switch (bm) {
    case BM_B1: return bm_ptr_b1(batched, dtype, vi);
    case BM_B3: return bm_ptr_b3(batched, dtype, vi);
    case BM_B2: return bm_ptr_b2(batched, dtype, vi);
    }
    return nullptr;
}

static bool polar_vi_ok(int vi) { return vi >= 0 && vi < kNPolar; }

static const void *polar_gen_ptr(int mode, int vm, int dtype, int vi)
{
    if (!polar_vi_ok(vi))
        return nullptr;
    switch (vm) {
    case VM_P: return polar_gen_ptr_p(mode, dtype, vi);
    case VM_P2: return polar_gen_ptr_p2(mode, dtype, vi);
    case VM_R:
        // trace mode: the masks and prefixes are the same for every value
        // method's generate kernel
        return mode == MODE_TRACE ? polar_gen_ptr_p(mode, dtype, vi) : polar_gen_ptr_r(mode, dtype, vi);
    }
    return nullptr;
}

static const void *polar_mask_ptr(int mode, int vm, int vi)
{
    if (!polar_vi_ok(vi))
        return nullptr;
    switch (vm) {
    case VM_P: return polar_mask_ptr_p(mode, vi);
    case VM_P2: return polar_mask_ptr_p2(mode, vi);
    case VM_R: return polar_mask_ptr_r(mode, vi);
    }
    return nullptr;
}

static const void *polar_scan_ptr(int mode)
{
    switch (mode) {
    case MODE_SINGLE: return (const void *)polar_scan_kernel<MODE_SINGLE>;
    case MODE_BATCHED: return (const void *)polar_scan_kernel<MODE_BATCHED>;
    case MODE_XY: return (const void *)polar_scan_kernel<MODE_XY>;
    case MODE_TRACE: return (const void *)polar_scan_kernel<MODE_TRACE>;
    }
    return nullptr;
}

static int launch_args(const void *fn, uint32_t grid, uint32_t block, void *argp, hipStream_t s,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    if (!fn)
        return (int)hipErrorInvalidValue;
    void *args[] = {argp};
    if (ev0 || ev1)   // the events take the dispatch's own start and end times
        return (int)hipExtLaunchKernel(fn, dim3(grid), dim3(block), args, 0, s, ev0, ev1, 0);
    return (int)hipLaunchKernel(fn, dim3(grid), dim3(block), args, 0, s);
}

int launch_b1_single(int bm, int dtype, int vi, const B1Args &a, uint32_t grid, hipStream_t s)
{
    B1Args c = a;
    return launch_args(b1_ptr(0, bm, dtype, vi), grid, kB1Variants[vi].wg, &c, s);
}

int launch_b1_batched(int bm, int dtype, int vi, const B1Args &a, uint32_t grid, hipStream_t s, hipEvent_t ev0,
                      hipEvent_t ev1)
{
    B1Args c = a;
    return launch_args(b1_ptr(1, bm, dtype, vi), grid, kB1Variants[vi].wg, &c, s, ev0, ev1);
}

int launch_b1_words(int bm, int dtype, const B1Args &a, uint64_t npairs, hipStream_t s)
{
    B1Args c = a;
    uint64_t np = npairs;
    void *args[] = {&c, &np};
    const void *fn = bm == BM_B3 ? bm_words_ptr_b3(dtype)
                                 : (bm == BM_B2 ? bm_words_ptr_b2(dtype) : bm_words_ptr_b1(dtype));
    if (!fn)
        return (int)hipErrorInvalidValue;
    uint64_t blocks = (npairs + 255) / 256;
    uint32_t grid = (uint32_t)(blocks < 65536 ? (blocks ? blocks : 1) : 65536);
    return (int)hipLaunchKernel(fn, dim3(grid), dim3(256), args, 0, s);
}

int launch_polar(int mode, int vm, int dtype, int vi, const PolarArgs &a, uint32_t grid_mask, uint32_t grid_gen,
                 hipStream_t s, int part, hipEvent_t ev0, hipEvent_t ev1)
{
    PolarArgs c = a;
    const void *gen = polar_gen_ptr(mode, vm, dtype, vi);
    if (!gen)
        return (int)hipErrorInvalidValue;
    int rc = (int)hipSuccess;
    if (part != 2) {
        rc = launch_args(polar_mask_ptr(mode, vm, vi), grid_mask, kMaskWG, &c, s);
        if (rc == (int)hipSuccess)
            rc = launch_args(polar_scan_ptr(mode), 1, 1024, &c, s);
    }
    if (rc == (int)hipSuccess && part != 1)
        rc = launch_args(gen, grid_gen, kPolarVariants[vi].wg, &c, s, ev0, ev1);
    return rc;
}

int launch_prep(const PrepArgs &a, hipStream_t s)
{
    PrepArgs c = a;
    return launch_args((const void *)prep_kernel, 1, 1024, &c, s);
}

int occupancy_polar(int mode, int vm, int dtype, int vi, int *blocks_per_cu)
{
    const void *fn = polar_gen_ptr(mode, vm, dtype, vi);
    if (!fn)
        return (int)hipErrorInvalidValue;
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, (int)kPolarVariants[vi].wg, 0);
}

int occupancy_polar_mask(int mode, int vm, int vi, int *blocks_per_cu)
{
    const void *fn = polar_mask_ptr(mode, vm, vi);
    if (!fn)
        return (int)hipErrorInvalidValue;
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, (int)kMaskWG, 0);
}

int occupancy_b1(int batched, int bm, int dtype, int vi, int *blocks_per_cu)
{
    const void *fn = b1_ptr(batched, bm, dtype, vi);
    if (!fn)
        return (int)hipErrorInvalidValue;
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, (int)kB1Variants[vi].wg, 0);
}

int launch_probe_store(void *out, uint64_t nbytes, uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(probe_store_kernel, dim3(grid), dim3(256), 0, s, (uint4 *)out, nbytes / 16);
    return (int)hipGetLastError();
}

int launch_probe_store_var(void *out, uint64_t nbytes, int nt, uint32_t unroll, uint32_t grid, hipStream_t s)
{
    const void *fn = nullptr;
    switch (unroll * 2 + (nt ? 1 : 0)) {
    case 2: fn = (const void *)probe_store_var_kernel<false, 1>; break;
    case 3: fn = (const void *)probe_store_var_kernel<true, 1>; break;
    case 4: fn = (const void *)probe_store_var_kernel<false, 2>; break;
    case 5: fn = (const void *)probe_store_var_kernel<true, 2>; break;
    case 8: fn = (const void *)probe_store_var_kernel<false, 4>; break;
    case 9: fn = (const void *)probe_store_var_kernel<true, 4>; break;
    case 16: fn = (const void *)probe_store_var_kernel<false, 8>; break;
    case 17: fn = (const void *)probe_store_var_kernel<true, 8>; break;
    }
    if (!fn)
        return (int)hipErrorInvalidValue;
    uint4 *o = (uint4 *)out;
    uint64_t n16 = nbytes / 16;
    void *args[] = {&o, &n16};
    return (int)hipLaunchKernel(fn, dim3(grid), dim3(256), args, 0, s);
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
