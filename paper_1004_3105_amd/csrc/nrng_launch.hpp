// nrng_launch.hpp -- internal interface between the C ABI (nrng_abi.cpp) and
// the kernels (nrng_kernels_*.hip).  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nrng {

enum Mode { MODE_SINGLE = 0, MODE_BATCHED = 1, MODE_TRACE = 2, MODE_XY = 3 };

// The Polar method runs as three kernels over tiles of 64 U candidates
// (U accept-mask words):
//   mask      hash, exact predicate and ballots of every candidate of the
//             budget; writes the mask words, each tile's accepted count as an
//             exclusive prefix within its chunk of kChunkTiles tiles, and the
//             chunk's total;
//   scan      one workgroup: exclusive prefix of the chunk totals;
//   generate  per tile, the accepted candidates are listed from the masks and
//             the lanes of a wave each take consecutive accepted pairs, so
//             that only accepted candidates are re-hashed and transformed and
//             the output is written with one 16-byte store per lane and pass.
// No kernel waits on another workgroup, and consecutive launches and graph
// replays need no clearing of the workspace.
constexpr uint32_t kChunkTiles = 16;
constexpr uint32_t kMaskWG = 256;

struct PolarArgs {
    // single stream / trace / xy
    uint64_t seed;
    uint64_t offset;
    uint64_t *cursor;        // device cursor (nullable): offset = *cursor, advanced by the consumed count
    uint64_t n;              // normals to produce (single); ignored for trace / xy
    uint64_t nwords;         // single / trace / xy: candidate budget in 64-candidate words
    uint64_t ntiles;         // single / trace / xy: tiles of the budget
    double mu, sigma;
    void *out;
    uint64_t *consumed;      // single: device pointer (nullable)
    // batched
    uint32_t nstreams;
    const uint64_t *tile_start;    // nstreams + 1 entries (built on the device by prep_kernel)
    const uint64_t *stream_words;  // nstreams entries: candidate budget of each stream, in words
    const uint64_t *seeds, *offsets, *ns, *out_off;
    const double *mus, *sigmas;
    uint64_t *consumed_arr;
    // workspace
    uint64_t *masks;         // accept-mask words, tile t's words at [t U, t U + U)
    uint32_t *ipfx;          // per tile: accepted pairs before it within its chunk
    uint32_t *tile_stream;   // batched, per tile: its stream (written by the mask kernel)
    uint32_t *csum;          // per chunk: accepted pairs in it
    uint64_t *cpfx;          // per chunk: accepted pairs before it (all streams together)
    uint64_t *misc;          // [0]: the single-stream offset read from *cursor by the scan kernel
    // trace / explicit candidates
    uint64_t ncand;
    uint64_t *word_prefix;
    const int32_t *xy;       // Polar, P2: explicit (X, Y) pairs
    const uint64_t *uvw;     // Algorithm R: explicit (u-word, v-word) pairs
    uint64_t *count_out;
    // Algorithm R: sqrt(8/e), rounded as the host computes it
    double ratio_c;
};

struct B1Args {
    uint64_t ctr0;           // seed + offset
    uint64_t n;
    double mu, sigma;
    void *out;
    const uint64_t *words;   // explicit hash words (test hook; 2 per pair for B1, 3 for B3) or null
    // batched
    uint32_t nstreams;
    const uint64_t *tile_start;
    const uint64_t *seeds, *offsets, *ns, *out_off;
    const double *mus, *sigmas;
};

// Batched Box-Muller family: a stream's output is cut into segments in
// virtual elements x = (stream element) + sh, with sh the even shift below one
// 128-byte line that puts x = 0 (and every pass, 64 groups of 16 bytes) on a
// line boundary of the output when the buffer itself is line-aligned.  The
// set-up kernel counts the tiles of a stream over n + sh elements.
constexpr uint64_t kLineBytes = 128;
__host__ __device__ inline uint64_t line_shift_elems(uint64_t off, uint64_t esize)
{
    return (off & (kLineBytes / esize - 1)) & ~1ull;
}

struct PrepArgs {
    int method;                      // 0 = B1, 1 = Polar, 2 = P2, 3 = B3, 4 = Algorithm R, 5 = B2
    uint32_t esize;                  // bytes per output element (Box-Muller family: the line shift)
    uint32_t nstreams;
    const uint64_t *ns, *out_off;    // out_off nullable (packed)
    uint64_t out_len;
    uint64_t unit;                   // B1, B3: pairs per tile; Polar, P2: mask words per tile
    uint64_t word_cap;               // Polar: workspace capacity in mask words (tiles x unit)
    uint64_t tile_cap;               // Polar: workspace capacity in tiles
    uint64_t *tile_start;            // out: nstreams + 1
    uint64_t *stream_words;          // out (Polar): nstreams, candidate budget in words
    uint64_t *packed_off;            // out: nstreams (used when out_off is null)
    uint64_t *consumed;              // out (nullable)
};

// Variant tables.
struct Variant { uint32_t wg, unroll; };
int b1_variants(const Variant **v);
int polar_variants(const Variant **v);

// Launchers (return hipError_t as int).  `vi` indexes the variant table.
// B1 family: bm 0 = Algorithm B1, 1 = method B3.
int launch_b1_single(int bm, int dtype, int vi, const B1Args &a, uint32_t grid, hipStream_t s);
int launch_b1_words(int bm, int dtype, const B1Args &a, uint64_t npairs, hipStream_t s);
// ev0 / ev1 (either may be null): events that record the batched kernel's
// own start and end (hipExtLaunchKernel), with no marker in the stream.
int launch_b1_batched(int bm, int dtype, int vi, const B1Args &a, uint32_t grid, hipStream_t s,
                      hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Polar: the mask, scan and generate kernels, in that order on stream s.
// vm selects the value method: 0 = Algorithm P, 1 = method P2 (no trace
// mode), 2 = Algorithm R (one output element per accepted candidate).
// grid_mask / grid_gen are the persistent grid sizes of the first and last.
// part 0 launches all three, 1 the mask and scan kernels, 2 the generate
// kernel; ev0 / ev1 as for launch_b1_batched, on the generate kernel.
int launch_polar(int mode, int vm, int dtype, int vi, const PolarArgs &a, uint32_t grid_mask, uint32_t grid_gen,
                 hipStream_t s, int part = 0, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
int launch_prep(const PrepArgs &a, hipStream_t s);

// Fixed device scratch of the allocation-free Polar entry point: its size,
// the largest n it serves, and its device address on device `dev` (which
// must be the current device), taken once per device with
// hipGetSymbolAddress and kept.  Returns a hipError_t as int.
constexpr uint64_t kScratchBytes = 8ull << 20;
constexpr uint64_t kScratchMaxN = 1ull << 26;
int scratch_address(int dev, void **addr);
int occupancy_polar(int mode, int vm, int dtype, int vi, int *blocks_per_cu);        // generate kernel
int occupancy_polar_mask(int mode, int vm, int vi, int *blocks_per_cu);
int occupancy_b1(int batched, int bm, int dtype, int vi, int *blocks_per_cu);
int launch_probe_store(void *out, uint64_t nbytes, uint32_t grid, hipStream_t s);
int launch_probe_store_var(void *out, uint64_t nbytes, int nt, uint32_t unroll, uint32_t grid, hipStream_t s);
int launch_probe_copy(void *dst, const void *src, uint64_t nbytes, uint32_t grid, hipStream_t s);
constexpr int kProbeValuOps = 15;   // instructions of the issue-rate probe (see nrng.h)
int launch_probe_valu(int op, uint32_t iters, uint32_t *sink, uint64_t sink_len, uint32_t grid, hipStream_t s);
int launch_probe_hash(uint64_t seed, uint64_t nhash, uint64_t *sink, uint64_t sink_len, uint32_t grid,
                      hipStream_t s);

// Candidate budget of a rejection stream that needs `need` accepted
// candidates at acceptance probability p, in words of 64 candidates: the
// expected candidate count need / p, plus four standard deviations of the
// negative-binomial count, plus 64.  Exceeding the budget is not an error
// (the stream's last tile continues serially past it); the budget only sizes
// the mask pass.
__host__ __device__ inline uint64_t candidate_budget_words(uint64_t need, double p)
{
    if (need == 0)
        return 0;
    const double q = 1.0 - p;
    const double P = (double)need;
    const double c = (P + 4.0 * sqrt(P * q)) / p + 64.0;
    return (uint64_t)(c * (1.0 / 64.0)) + 1;
}

// Polar and P2: one accepted candidate per pair, p = pi/4.
constexpr double kPolarAccept = 0.78539816339744830962;
// Algorithm R: one accepted candidate per normal, p = sqrt(pi e)/4.
constexpr double kRatioAccept = 0.73057059133056956;

__host__ __device__ inline uint64_t polar_budget_words(uint64_t npairs)
{
    return candidate_budget_words(npairs, kPolarAccept);
}

// Budget of a stream of n normals for PrepArgs / PolarArgs method ids 1
// (Polar), 2 (P2) and 4 (Algorithm R).
__host__ __device__ inline uint64_t method_budget_words(int method, uint64_t n)
{
    return method == 4 ? candidate_budget_words(n, kRatioAccept) : polar_budget_words((n + 1) / 2);
}

}  // namespace nrng
