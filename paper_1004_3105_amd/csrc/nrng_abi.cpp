// nrng_abi.cpp -- the C ABI of libnrng.so (declared in include/nrng.h):
// argument validation, the per-device workspace, launch configuration and
// dispatch to the kernels in nrng_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "../../include/nrng.h"
#include "nrng_launch.hpp"

using namespace nrng;

namespace {

constexpr int kMaxDev = 64;

struct DevState {
    bool init = false;
    int cus = 0;
    Ctl *ctl = nullptr;
    uint64_t *status = nullptr;
    uint64_t status_cap = 0;
    uint64_t *bst = nullptr;        // block status words
    uint64_t bcap = 0;
    uint64_t *tile_start = nullptr;
    uint64_t *block_start = nullptr;
    uint64_t *packed_off = nullptr;
    uint64_t stream_cap = 0;
    int occ_polar[4][4][8] = {};     // [mode][dtype][variant], 0 = not queried
    int occ_b1[2][4][8] = {};        // [batched][dtype][variant]
    // the tile table currently in the workspace (from nrng_batched_plan)
    int plan_method = -1, plan_dtype = -1, plan_vi = -1;
    uint32_t plan_nstreams = 0;
    bool plan_packed = false;
};

struct Tune {
    int vi;
    uint32_t grid_per_cu;
};

std::mutex g_mu;
DevState g_dev[kMaxDev];
// Defaults chosen by the autotuner on MI355X (see the tune table written by
// the Python autotuner); kernel ids: 0 = B1 single, 1 = Polar, 2 = B1 batched.
Tune g_tune[3][4] = {
    {{1, 0}, {1, 0}, {1, 0}, {1, 0}},
    {{1, 0}, {1, 0}, {1, 0}, {1, 0}},
    {{1, 0}, {1, 0}, {1, 0}, {1, 0}},
};

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

bool dtype_ok(int d) { return d >= NRNG_F64 && d <= NRNG_F16; }

int check_mu_sigma(double mu, double sigma)
{
    if (!std::isfinite(mu) || !std::isfinite(sigma) || sigma < 0.0)
        return NRNG_EINVAL;
    return NRNG_OK;
}

int hip_status(int e)
{
    return e == (int)hipSuccess ? NRNG_OK : NRNG_EHIP;
}

bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess)
        return false;
    return st != hipStreamCaptureStatusNone;
}

// Current device's state, initialised on first use.  Caller holds g_mu.
int get_dev(DevState **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev)
        return NRNG_ENODEV;
    DevState &d = g_dev[dev];
    if (!d.init) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
            return NRNG_ENODEV;
        d.cus = prop.multiProcessorCount;
        if (hipMalloc(&d.ctl, sizeof(Ctl)) != hipSuccess)
            return NRNG_ENOMEM;
        Ctl c0 = {0, 0, 1, 0, 0};
        if (hipMemcpy(d.ctl, &c0, sizeof(Ctl), hipMemcpyHostToDevice) != hipSuccess)
            return NRNG_EHIP;
        d.init = true;
    }
    *out = &d;
    return NRNG_OK;
}

// Grow the look-back arrays to at least `tiles` tile words and `blocks`
// block words (all zeroed).
int ensure_status(DevState &d, uint64_t tiles, uint64_t blocks, hipStream_t s)
{
    if (tiles <= d.status_cap && blocks <= d.bcap)
        return NRNG_OK;
    if (capturing(s))
        return NRNG_ECAPTURE;
    if (tiles > (1ull << 36) || blocks > (1ull << 36))
        return NRNG_ERANGE;
    const uint64_t cap = std::max<uint64_t>(tiles + tiles / 4 + 1024, d.status_cap);
    const uint64_t bcap = std::max<uint64_t>(blocks + blocks / 4 + 256, d.bcap);
    if (hipDeviceSynchronize() != hipSuccess)
        return NRNG_EHIP;
    for (uint64_t **p : {&d.status, &d.bst}) {
        if (*p)
            hipFree(*p);
        *p = nullptr;
    }
    d.status_cap = d.bcap = 0;
    const size_t sb = cap * kStatusStride * sizeof(uint64_t), bb = bcap * kStatusStride * sizeof(uint64_t);
    if (hipMalloc(&d.status, sb) != hipSuccess || hipMalloc(&d.bst, bb) != hipSuccess)
        return NRNG_ENOMEM;
    if (hipMemset(d.status, 0, sb) != hipSuccess || hipMemset(d.bst, 0, bb) != hipSuccess)
        return NRNG_EHIP;
    if (hipDeviceSynchronize() != hipSuccess)
        return NRNG_EHIP;
    d.status_cap = cap;
    d.bcap = bcap;
    return NRNG_OK;
}

int ensure_streams(DevState &d, uint64_t nstreams, hipStream_t s)
{
    if (nstreams <= d.stream_cap)
        return NRNG_OK;
    if (capturing(s))
        return NRNG_ECAPTURE;
    uint64_t cap = nstreams + nstreams / 4 + 256;
    if (hipDeviceSynchronize() != hipSuccess)
        return NRNG_EHIP;
    for (uint64_t **p : {&d.tile_start, &d.block_start, &d.packed_off}) {
        if (*p)
            hipFree(*p);
        *p = nullptr;
    }
    d.stream_cap = 0;
    if (hipMalloc(&d.tile_start, (cap + 1) * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc(&d.block_start, (cap + 1) * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc(&d.packed_off, cap * sizeof(uint64_t)) != hipSuccess)
        return NRNG_ENOMEM;
    d.stream_cap = cap;
    return NRNG_OK;
}

int polar_blocks_per_cu(DevState &d, int mode, int dtype, int vi)
{
    int &o = d.occ_polar[mode][dtype][vi];
    if (o == 0) {
        int b = 0;
        if (occupancy_polar(mode, dtype, vi, &b) != (int)hipSuccess || b <= 0)
            b = 1;
        o = b;
    }
    return o;
}

int b1_blocks_per_cu(DevState &d, int batched, int dtype, int vi)
{
    int &o = d.occ_b1[batched][dtype][vi];
    if (o == 0) {
        int b = 0;
        if (occupancy_b1(batched, dtype, vi, &b) != (int)hipSuccess || b <= 0)
            b = 1;
        o = b;
    }
    return o;
}

uint32_t persistent_grid(DevState &d, int per_cu_occ, uint32_t per_cu_cap, uint64_t need)
{
    uint64_t per = per_cu_cap ? (per_cu_cap < (uint32_t)per_cu_occ ? per_cu_cap : (uint32_t)per_cu_occ)
                              : (uint32_t)per_cu_occ;
    uint64_t g = (uint64_t)d.cus * per;
    if (need && need < g)
        g = need;
    if (g < 1)
        g = 1;
    if (g > 0x7FFFFFFF)
        g = 0x7FFFFFFF;
    return (uint32_t)g;
}

// Candidates per Polar tile: one wave's 64 lanes times the unroll.
uint64_t polar_tile_cand(int vi)
{
    const Variant *v;
    polar_variants(&v);
    return 64ull * v[vi].unroll;
}

// Upper bound on the batched Polar tile count when the valid streams hold
// at most out_len normals: each stream of P >= 1 pairs has at most
// (3.6346 P + 64) / C + 1 tiles (see polar_budget_tiles).
uint64_t batched_polar_tile_bound(uint64_t out_len, uint64_t nstreams, uint64_t C)
{
    const double pairs = ((double)out_len + (double)nstreams) / 2.0;
    const double b = (3.6346 * pairs + 64.0 * (double)nstreams) / (double)C + (double)nstreams + 2.0;
    if (b > 1.0e15)
        return ~0ull;
    return (uint64_t)b;
}

int polar_common(int mode, uint64_t seed, uint64_t offset, uint64_t *cursor, uint64_t n, double mu, double sigma,
                 void *out, int dtype, hipStream_t s, uint64_t *d_consumed, uint32_t force_tiles)
{
    if (!dtype_ok(dtype))
        return NRNG_EDTYPE;
    int rc = check_mu_sigma(mu, sigma);
    if (rc)
        return rc;
    if (n == 0)
        return NRNG_OK;
    if (!out)
        return NRNG_EINVAL;
    if (n > (1ull << 41))
        return NRNG_ERANGE;
    std::lock_guard<std::mutex> lk(g_mu);
    DevState *d;
    if ((rc = get_dev(&d)))
        return rc;
    const Tune tu = g_tune[1][dtype];
    const uint64_t C = polar_tile_cand(tu.vi);
    uint64_t tiles = force_tiles ? force_tiles : polar_budget_tiles((n + 1) / 2, C);
    if (tiles >= (1ull << 31))
        return NRNG_ERANGE;
    if ((rc = ensure_status(*d, tiles, (tiles + 63) / 64, s)))
        return rc;
    PolarArgs a;
    std::memset(&a, 0, sizeof(a));
    a.seed = seed;
    a.offset = offset;
    a.cursor = cursor;
    a.n = n;
    a.ntiles = (uint32_t)tiles;
    a.mu = mu;
    a.sigma = sigma;
    a.out = out;
    a.consumed = d_consumed;
    a.status = d->status;
    a.status_cap = d->status_cap;
    a.bst = d->bst;
    a.bcap = d->bcap;
    a.ctl = d->ctl;
    const uint32_t grid = persistent_grid(*d, polar_blocks_per_cu(*d, mode, dtype, tu.vi), tu.grid_per_cu, tiles);
    return hip_status(launch_polar(mode, dtype, tu.vi, a, grid, s));
}

}  // namespace

extern "C" {

const char *nrng_strerror(int status)
{
    switch (status) {
    case NRNG_OK: return "success";
    case NRNG_EINVAL: return "invalid argument";
    case NRNG_EDTYPE: return "unknown dtype";
    case NRNG_ERANGE: return "size out of range";
    case NRNG_EHIP: return "HIP runtime error";
    case NRNG_ENODEV: return "no usable GPU";
    case NRNG_ECAPTURE: return "workspace growth needed during stream capture (call nrng_reserve first)";
    case NRNG_ENOMEM: return "device allocation failed";
    }
    return "unknown status";
}

int nrng_version(void) { return 10000; }

int nrng_init(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    DevState *d;
    return get_dev(&d);
}

int nrng_device_cus(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    DevState *d;
    if (get_dev(&d))
        return 0;
    return d->cus;
}

int nrng_reserve(uint64_t max_n, uint32_t max_streams)
{
    std::lock_guard<std::mutex> lk(g_mu);
    DevState *d;
    int rc = get_dev(&d);
    if (rc)
        return rc;
    // the smallest tile of any variant gives the largest tile count
    const Variant *v;
    const int nv = polar_variants(&v);
    uint64_t cmin = ~0ull;
    for (int i = 0; i < nv; ++i)
        cmin = std::min<uint64_t>(cmin, 64ull * v[i].unroll);
    uint64_t tiles = polar_budget_tiles((max_n + 1) / 2, cmin);
    if (max_streams)
        tiles = std::max<uint64_t>(tiles, batched_polar_tile_bound(max_n, max_streams, cmin));
    if ((rc = ensure_status(*d, tiles, tiles / 64 + max_streams + 1, nullptr)))
        return rc;
    if (max_streams && (rc = ensure_streams(*d, max_streams, nullptr)))
        return rc;
    return NRNG_OK;
}

int nrng_boxmuller(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, void *out, int dtype,
                   void *stream)
{
    if (!dtype_ok(dtype))
        return NRNG_EDTYPE;
    int rc = check_mu_sigma(mu, sigma);
    if (rc)
        return rc;
    if (n == 0)
        return NRNG_OK;
    if (!out)
        return NRNG_EINVAL;
    if (n > (1ull << 62))
        return NRNG_ERANGE;
    std::lock_guard<std::mutex> lk(g_mu);
    DevState *d;
    if ((rc = get_dev(&d)))
        return rc;
    const Tune tu = g_tune[0][dtype];
    const Variant *v;
    b1_variants(&v);
    const uint64_t ppl = (dtype == NRNG_F64) ? 1 : (dtype == NRNG_F32 ? 2 : 4);
    const uint64_t nchunks = ((n + 1) / 2 + ppl - 1) / ppl;
    const uint64_t blocks = (nchunks + (uint64_t)v[tu.vi].wg * v[tu.vi].unroll - 1) /
                            ((uint64_t)v[tu.vi].wg * v[tu.vi].unroll);
    const uint32_t grid = persistent_grid(*d, b1_blocks_per_cu(*d, 0, dtype, tu.vi), tu.grid_per_cu, blocks);
    B1Args a;
    std::memset(&a, 0, sizeof(a));
    a.ctr0 = seed + offset;
    a.n = n;
    a.mu = mu;
    a.sigma = sigma;
    a.out = out;
    return hip_status(launch_b1_single(dtype, tu.vi, a, grid, S(stream)));
}

int nrng_polar(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, void *out, int dtype,
               void *stream, uint64_t *d_consumed)
{
    return polar_common(MODE_SINGLE, seed, offset, nullptr, n, mu, sigma, out, dtype, S(stream), d_consumed, 0);
}

int nrng_polar_dev(uint64_t seed, uint64_t *d_cursor, uint64_t n, double mu, double sigma, void *out, int dtype,
                   void *stream)
{
    if (!d_cursor)
        return NRNG_EINVAL;
    return polar_common(MODE_SINGLE, seed, 0, d_cursor, n, mu, sigma, out, dtype, S(stream), nullptr, 0);
}

int nrng_test_polar_budget(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, void *out,
                           int dtype, uint32_t tiles, void *stream, uint64_t *d_consumed)
{
    if (tiles == 0)
        return NRNG_EINVAL;
    return polar_common(MODE_SINGLE, seed, offset, nullptr, n, mu, sigma, out, dtype, S(stream), d_consumed,
                        tiles);
}

int nrng_batched_plan(int method, uint32_t nstreams, const uint64_t *d_n, const uint64_t *d_out_off,
                      uint64_t out_len, int dtype, void *stream, uint64_t *d_consumed)
{
    if (!dtype_ok(dtype))
        return NRNG_EDTYPE;
    if (method != NRNG_METHOD_B1 && method != NRNG_METHOD_POLAR)
        return NRNG_EINVAL;
    if (nstreams == 0)
        return NRNG_OK;
    if (!d_n)
        return NRNG_EINVAL;
    if (out_len > (1ull << 41))
        return NRNG_ERANGE;
    hipStream_t s = S(stream);
    std::lock_guard<std::mutex> lk(g_mu);
    DevState *d;
    int rc = get_dev(&d);
    if (rc)
        return rc;
    if ((rc = ensure_streams(*d, nstreams, s)))
        return rc;
    const int kid = method == NRNG_METHOD_B1 ? 2 : 1;
    const Tune tu = g_tune[kid][dtype];
    PrepArgs p;
    std::memset(&p, 0, sizeof(p));
    p.method = method;
    p.nstreams = nstreams;
    p.ns = d_n;
    p.out_off = d_out_off;
    p.out_len = out_len;
    p.tile_start = d->tile_start;
    p.packed_off = d->packed_off;
    p.consumed = d_consumed;
    if (method == NRNG_METHOD_B1) {
        const Variant *v;
        b1_variants(&v);
        const uint64_t ppl = (dtype == NRNG_F64) ? 1 : (dtype == NRNG_F32 ? 2 : 4);
        p.unit = (uint64_t)v[tu.vi].wg * v[tu.vi].unroll * ppl;
    } else {
        const uint64_t C = polar_tile_cand(tu.vi);
        const uint64_t bound = batched_polar_tile_bound(out_len, nstreams, C);
        if (bound == ~0ull)
            return NRNG_ERANGE;
        if ((rc = ensure_status(*d, bound, bound / 64 + nstreams + 1, s)))
            return rc;
        p.unit = C;
        p.status_cap = d->status_cap;
        p.block_cap = d->bcap;
        p.block_start = d->block_start;
    }
    if ((rc = hip_status(launch_prep(p, s))))
        return rc;
    d->plan_method = method;
    d->plan_dtype = dtype;
    d->plan_vi = tu.vi;
    d->plan_nstreams = nstreams;
    d->plan_packed = d_out_off == nullptr;
    return NRNG_OK;
}

int nrng_batched_exec(int method, uint32_t nstreams, const uint64_t *d_seed, const uint64_t *d_offset,
                      const uint64_t *d_n, const uint64_t *d_out_off, const double *d_mu, const double *d_sigma,
                      void *out, int dtype, void *stream, uint64_t *d_consumed)
{
    if (!dtype_ok(dtype))
        return NRNG_EDTYPE;
    if (method != NRNG_METHOD_B1 && method != NRNG_METHOD_POLAR)
        return NRNG_EINVAL;
    if (nstreams == 0)
        return NRNG_OK;
    if (!d_seed || !d_offset || !d_n || !d_mu || !d_sigma)
        return NRNG_EINVAL;
    hipStream_t s = S(stream);
    std::lock_guard<std::mutex> lk(g_mu);
    DevState *d;
    int rc = get_dev(&d);
    if (rc)
        return rc;
    // the tile table must come from a plan for this method, dtype, variant,
    // stream count and layout
    const int kid = method == NRNG_METHOD_B1 ? 2 : 1;
    const Tune tu = g_tune[kid][dtype];
    if (d->plan_method != method || d->plan_dtype != dtype || d->plan_vi != tu.vi ||
        d->plan_nstreams != nstreams || d->plan_packed != (d_out_off == nullptr))
        return NRNG_EINVAL;
    if (!out)
        return NRNG_EINVAL;
    const uint64_t *off = d_out_off ? d_out_off : d->packed_off;
    if (method == NRNG_METHOD_B1) {
        B1Args a;
        std::memset(&a, 0, sizeof(a));
        a.out = out;
        a.nstreams = nstreams;
        a.tile_start = d->tile_start;
        a.seeds = d_seed;
        a.offsets = d_offset;
        a.ns = d_n;
        a.out_off = off;
        a.mus = d_mu;
        a.sigmas = d_sigma;
        const uint32_t grid = persistent_grid(*d, b1_blocks_per_cu(*d, 1, dtype, tu.vi), tu.grid_per_cu, 0);
        return hip_status(launch_b1_batched(dtype, tu.vi, a, grid, s));
    }
    PolarArgs a;
    std::memset(&a, 0, sizeof(a));
    a.mu = 0.0;
    a.sigma = 1.0;
    a.out = out;
    a.nstreams = nstreams;
    a.tile_start = d->tile_start;
    a.seeds = d_seed;
    a.offsets = d_offset;
    a.ns = d_n;
    a.out_off = off;
    a.mus = d_mu;
    a.sigmas = d_sigma;
    a.consumed_arr = d_consumed;
    a.block_start = d->block_start;
    a.status = d->status;
    a.status_cap = d->status_cap;
    a.bst = d->bst;
    a.bcap = d->bcap;
    a.ctl = d->ctl;
    const uint32_t grid =
        persistent_grid(*d, polar_blocks_per_cu(*d, MODE_BATCHED, dtype, tu.vi), tu.grid_per_cu, 0);
    return hip_status(launch_polar(MODE_BATCHED, dtype, tu.vi, a, grid, s));
}

int nrng_batched(int method, uint32_t nstreams, const uint64_t *d_seed, const uint64_t *d_offset,
                 const uint64_t *d_n, const uint64_t *d_out_off, const double *d_mu, const double *d_sigma,
                 void *out, uint64_t out_len, int dtype, void *stream, uint64_t *d_consumed)
{
    if (!dtype_ok(dtype))
        return NRNG_EDTYPE;
    if (method != NRNG_METHOD_B1 && method != NRNG_METHOD_POLAR)
        return NRNG_EINVAL;
    if (nstreams == 0)
        return NRNG_OK;
    if (!d_seed || !d_offset || !d_n || !d_mu || !d_sigma)
        return NRNG_EINVAL;
    if (!out && out_len > 0)
        return NRNG_EINVAL;
    int rc = nrng_batched_plan(method, nstreams, d_n, d_out_off, out_len, dtype, stream, d_consumed);
    if (rc)
        return rc;
    if (!out)
        return NRNG_OK;   // out_len == 0: every stream with n > 0 was skipped by the plan
    return nrng_batched_exec(method, nstreams, d_seed, d_offset, d_n, d_out_off, d_mu, d_sigma, out, dtype, stream,
                             d_consumed);
}

struct FillGraph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

int nrng_fillgraph_create(uint64_t seed, uint64_t *d_cursor, uint64_t n, double mu, double sigma, void *out,
                          int dtype, void *stream, void **graph)
{
    if (!graph || !d_cursor)
        return NRNG_EINVAL;
    *graph = nullptr;
    if (!dtype_ok(dtype))
        return NRNG_EDTYPE;
    int rc = check_mu_sigma(mu, sigma);
    if (rc)
        return rc;
    if (n == 0 || !out)
        return NRNG_EINVAL;
    hipStream_t s = S(stream);
    if (!s || capturing(s))
        return NRNG_EINVAL;
    if ((rc = nrng_reserve(n, 0)))
        return rc;
    FillGraph *g = new FillGraph();
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        delete g;
        return NRNG_EHIP;
    }
    rc = nrng_polar_dev(seed, d_cursor, n, mu, sigma, out, dtype, stream);
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &gr);
    if (rc || e != hipSuccess || !gr) {
        if (gr)
            hipGraphDestroy(gr);
        delete g;
        return rc ? rc : NRNG_EHIP;
    }
    g->graph = gr;
    if (hipGraphInstantiate(&g->exec, gr, nullptr, nullptr, 0) != hipSuccess) {
        hipGraphDestroy(gr);
        delete g;
        return NRNG_EHIP;
    }
    *graph = g;
    return NRNG_OK;
}

int nrng_fillgraph_launch(void *graph, void *stream)
{
    if (!graph)
        return NRNG_EINVAL;
    FillGraph *g = static_cast<FillGraph *>(graph);
    return hipGraphLaunch(g->exec, S(stream)) == hipSuccess ? NRNG_OK : NRNG_EHIP;
}

int nrng_fillgraph_destroy(void *graph)
{
    if (!graph)
        return NRNG_OK;
    FillGraph *g = static_cast<FillGraph *>(graph);
    hipGraphExecDestroy(g->exec);
    hipGraphDestroy(g->graph);
    delete g;
    return NRNG_OK;
}

int nrng_tune_set(int kernel, int dtype, uint32_t wg, uint32_t unroll, uint32_t grid_per_cu)
{
    if (kernel < 0 || kernel > 2)
        return NRNG_EINVAL;
    if (!dtype_ok(dtype))
        return NRNG_EDTYPE;
    const Variant *v;
    const int nv = kernel == 1 ? polar_variants(&v) : b1_variants(&v);
    for (int i = 0; i < nv; ++i) {
        if (v[i].wg == wg && v[i].unroll == unroll) {
            std::lock_guard<std::mutex> lk(g_mu);
            g_tune[kernel][dtype] = {i, grid_per_cu};
            return NRNG_OK;
        }
    }
    return NRNG_EINVAL;
}

int nrng_tune_get(int kernel, int dtype, uint32_t *wg, uint32_t *unroll, uint32_t *grid_per_cu)
{
    if (kernel < 0 || kernel > 2)
        return NRNG_EINVAL;
    if (!dtype_ok(dtype))
        return NRNG_EDTYPE;
    const Variant *v;
    kernel == 1 ? polar_variants(&v) : b1_variants(&v);
    std::lock_guard<std::mutex> lk(g_mu);
    const Tune t = g_tune[kernel][dtype];
    if (wg)
        *wg = v[t.vi].wg;
    if (unroll)
        *unroll = v[t.vi].unroll;
    if (grid_per_cu)
        *grid_per_cu = t.grid_per_cu;
    return NRNG_OK;
}

int nrng_tune_variants(int kernel, uint32_t *pairs, int max_pairs)
{
    if (kernel < 0 || kernel > 2)
        return NRNG_EINVAL;
    const Variant *v;
    const int nv = kernel == 1 ? polar_variants(&v) : b1_variants(&v);
    for (int i = 0; i < nv && i < max_pairs && pairs; ++i) {
        pairs[2 * i] = v[i].wg;
        pairs[2 * i + 1] = v[i].unroll;
    }
    return nv;
}

int nrng_test_b1_words(const uint64_t *d_words, uint64_t npairs, double mu, double sigma, void *out, int dtype,
                       void *stream)
{
    if (!dtype_ok(dtype))
        return NRNG_EDTYPE;
    int rc = check_mu_sigma(mu, sigma);
    if (rc)
        return rc;
    if (npairs == 0)
        return NRNG_OK;
    if (!d_words || !out)
        return NRNG_EINVAL;
    B1Args a;
    std::memset(&a, 0, sizeof(a));
    a.mu = mu;
    a.sigma = sigma;
    a.out = out;
    a.words = d_words;
    return hip_status(launch_b1_words(dtype, a, npairs, S(stream)));
}

int nrng_test_polar_xy(const int32_t *d_xy, uint64_t ncand, double mu, double sigma, void *out, int dtype,
                       uint64_t *d_mask_words, uint64_t *d_count, void *stream)
{
    if (!dtype_ok(dtype))
        return NRNG_EDTYPE;
    int rc = check_mu_sigma(mu, sigma);
    if (rc)
        return rc;
    if (ncand == 0)
        return NRNG_OK;
    if (!d_xy || !out || !d_mask_words || !d_count)
        return NRNG_EINVAL;
    hipStream_t s = S(stream);
    std::lock_guard<std::mutex> lk(g_mu);
    DevState *d;
    if ((rc = get_dev(&d)))
        return rc;
    const Tune tu = g_tune[1][dtype];
    const uint64_t C = polar_tile_cand(tu.vi);
    const uint64_t tiles = (ncand + C - 1) / C;
    if (tiles >= (1ull << 31))
        return NRNG_ERANGE;
    if ((rc = ensure_status(*d, tiles, (tiles + 63) / 64, s)))
        return rc;
    PolarArgs a;
    std::memset(&a, 0, sizeof(a));
    a.ntiles = (uint32_t)tiles;
    a.mu = mu;
    a.sigma = sigma;
    a.out = out;
    a.status = d->status;
    a.status_cap = d->status_cap;
    a.bst = d->bst;
    a.bcap = d->bcap;
    a.ctl = d->ctl;
    a.ncand = ncand;
    a.masks = d_mask_words;
    a.word_prefix = nullptr;
    a.xy = d_xy;
    a.count_out = d_count;
    const uint32_t grid = persistent_grid(*d, polar_blocks_per_cu(*d, MODE_XY, dtype, tu.vi), tu.grid_per_cu, tiles);
    return hip_status(launch_polar(MODE_XY, dtype, tu.vi, a, grid, s));
}

int nrng_polar_trace(uint64_t seed, uint64_t offset, uint64_t ncand, uint64_t *d_mask_words,
                     uint64_t *d_word_prefix, void *stream)
{
    if (ncand == 0)
        return NRNG_OK;
    if (!d_mask_words || !d_word_prefix)
        return NRNG_EINVAL;
    hipStream_t s = S(stream);
    std::lock_guard<std::mutex> lk(g_mu);
    DevState *d;
    int rc = get_dev(&d);
    if (rc)
        return rc;
    const Tune tu = g_tune[1][NRNG_F32];
    const uint64_t C = polar_tile_cand(tu.vi);
    const uint64_t tiles = (ncand + C - 1) / C;
    if (tiles >= (1ull << 31))
        return NRNG_ERANGE;
    if ((rc = ensure_status(*d, tiles, (tiles + 63) / 64, s)))
        return rc;
    PolarArgs a;
    std::memset(&a, 0, sizeof(a));
    a.seed = seed;
    a.offset = offset;
    a.ntiles = (uint32_t)tiles;
    a.mu = 0.0;
    a.sigma = 1.0;
    a.status = d->status;
    a.status_cap = d->status_cap;
    a.bst = d->bst;
    a.bcap = d->bcap;
    a.ctl = d->ctl;
    a.ncand = ncand;
    a.masks = d_mask_words;
    a.word_prefix = d_word_prefix;
    const uint32_t grid =
        persistent_grid(*d, polar_blocks_per_cu(*d, MODE_TRACE, NRNG_F32, tu.vi), tu.grid_per_cu, tiles);
    return hip_status(launch_polar(MODE_TRACE, NRNG_F32, tu.vi, a, grid, s));
}

int nrng_probe_store(void *out, uint64_t nbytes, void *stream)
{
    if (!out || nbytes % 16)
        return NRNG_EINVAL;
    if (nbytes == 0)
        return NRNG_OK;
    DevState *d;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        int rc = get_dev(&d);
        if (rc)
            return rc;
    }
    return hip_status(launch_probe_store(out, nbytes, (uint32_t)d->cus * 32, S(stream)));
}

int nrng_probe_copy(void *dst, const void *src, uint64_t nbytes, void *stream)
{
    if (!dst || !src || nbytes % 16)
        return NRNG_EINVAL;
    if (nbytes == 0)
        return NRNG_OK;
    DevState *d;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        int rc = get_dev(&d);
        if (rc)
            return rc;
    }
    return hip_status(launch_probe_copy(dst, src, nbytes, (uint32_t)d->cus * 32, S(stream)));
}

int nrng_probe_hash(uint64_t seed, uint64_t nhash, uint64_t *d_sink, uint64_t sink_len, void *stream)
{
    if (!d_sink || sink_len == 0)
        return NRNG_EINVAL;
    DevState *d;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        int rc = get_dev(&d);
        if (rc)
            return rc;
    }
    uint64_t grid = (uint64_t)d->cus * 8;
    return hip_status(launch_probe_hash(seed, nhash, d_sink, sink_len, (uint32_t)grid, S(stream)));
}

}  // extern "C"
