// nrng_launch.hpp -- internal interface between the C ABI (nrng_abi.cpp) and
// the kernels (nrng_kernels.hip).  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nrng {

// Per-device control block of the look-back kernels.  It resets itself at
// the end of every launch (the last workgroup to exit clears the exit
// counter and advances the epoch), so consecutive launches and graph replays
// need no memset.
struct Ctl {
    uint32_t unused;
    uint32_t exited;     // workgroups that have finished
    uint32_t epoch;      // tag of this launch's status words, 1 .. 2^22 - 1
    uint32_t pad;
    uint64_t consumed;   // single stream: uniforms consumed (for the cursor)
};

constexpr uint32_t kEpochLimit = 1u << 22;

// Status words (tile and block) are spaced kStatusStride words apart, so that
// the words of the tiles in flight at one moment spread over many memory
// channels instead of sharing a few cache lines.
#ifndef NRNG_STATUS_STRIDE
#define NRNG_STATUS_STRIDE 1
#endif
constexpr uint64_t kStatusStride = NRNG_STATUS_STRIDE;

enum Mode { MODE_SINGLE = 0, MODE_BATCHED = 1, MODE_TRACE = 2, MODE_XY = 3 };

struct PolarArgs {
    // single stream / trace
    uint64_t seed;
    uint64_t offset;
    uint64_t *cursor;        // device cursor (nullable): offset = *cursor, advanced at the end
    uint64_t n;              // normals to produce (single); ignored for trace / xy
    uint32_t ntiles;         // single / trace / xy: look-back tile budget
    double mu, sigma;
    void *out;
    uint64_t *consumed;      // single: device pointer (nullable)
    // batched
    uint32_t nstreams;
    const uint64_t *tile_start;   // nstreams + 1 entries (workspace, built on the device)
    const uint64_t *seeds, *offsets, *ns, *out_off;
    const double *mus, *sigmas;
    uint64_t *consumed_arr;
    const uint64_t *block_start;  // batched: nstreams + 1 entries, first block of each stream
    // workspace
    uint64_t *status;
    uint64_t status_cap;
    uint64_t *bst;           // block status words (tagged), bcap entries
    uint64_t bcap;
    Ctl *ctl;
    // trace / explicit candidates
    uint64_t ncand;
    uint64_t *masks, *word_prefix;
    const int32_t *xy;
    uint64_t *count_out;
};

struct B1Args {
    uint64_t ctr0;           // seed + offset
    uint64_t n;
    double mu, sigma;
    void *out;
    const uint64_t *words;   // explicit hash words (test hook) or null
    // batched
    uint32_t nstreams;
    const uint64_t *tile_start;
    const uint64_t *seeds, *offsets, *ns, *out_off;
    const double *mus, *sigmas;
};

struct PrepArgs {
    int method;
    uint32_t nstreams;
    const uint64_t *ns, *out_off;    // out_off nullable (packed)
    uint64_t out_len;
    uint64_t unit;                   // B1: pairs per tile; Polar: candidates per tile
    uint64_t status_cap;             // Polar: capacity in tiles
    uint64_t block_cap;              // Polar: capacity in blocks of 64 tiles
    uint64_t *tile_start;            // out: nstreams + 1
    uint64_t *block_start;           // out (Polar): nstreams + 1
    uint64_t *packed_off;            // out: nstreams (used when out_off is null)
    uint64_t *consumed;              // out (nullable)
};

// Variant tables.
struct Variant { uint32_t wg, unroll; };
int b1_variants(const Variant **v);
int polar_variants(const Variant **v);

// Launchers (return hipError_t as int).  `vi` indexes the variant table.
int launch_b1_single(int dtype, int vi, const B1Args &a, uint32_t grid, hipStream_t s);
int launch_b1_words(int dtype, const B1Args &a, uint64_t npairs, hipStream_t s);
int launch_b1_batched(int dtype, int vi, const B1Args &a, uint32_t grid, hipStream_t s);
int launch_polar(int mode, int dtype, int vi, const PolarArgs &a, uint32_t grid, hipStream_t s);
int launch_prep(const PrepArgs &a, hipStream_t s);
int occupancy_polar(int mode, int dtype, int vi, int *blocks_per_cu);
int occupancy_b1(int batched, int dtype, int vi, int *blocks_per_cu);
int launch_probe_store(void *out, uint64_t nbytes, uint32_t grid, hipStream_t s);
int launch_probe_copy(void *dst, const void *src, uint64_t nbytes, uint32_t grid, hipStream_t s);
int launch_probe_hash(uint64_t seed, uint64_t nhash, uint64_t *sink, uint64_t sink_len, uint32_t grid,
                      hipStream_t s);

// Tiles of the Polar look-back budget for a stream of npairs accepted pairs,
// with `cand` candidates per tile: the expected candidate count
// npairs / (pi/4), plus four standard deviations of the negative-binomial
// count, plus 64.  Exceeding the budget is not an error (the last tile of
// the stream continues serially); the budget only sizes the look-back.
__host__ __device__ inline uint64_t polar_budget_tiles(uint64_t npairs, uint64_t cand)
{
    if (npairs == 0)
        return 0;
    const double p = 0.78539816339744830962, q = 1.0 - p;
    const double P = (double)npairs;
    const double c = P / p + 4.0 * sqrt(P * q) / p + 64.0;
    uint64_t t = (uint64_t)(c / (double)cand) + 1;
    return t;
}

}  // namespace nrng
