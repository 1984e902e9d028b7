/*
 * nrng.h -- C ABI of libnrng.so: normal random deviates on AMD Instinct
 * MI355X (gfx950).
 *
 * The library turns a counter-based stream of uniform deviates into
 * N(mu, sigma^2) deviates by the two methods of Section 2 of R. P. Brent,
 * "Fast Normal Random Number Generators for Vector Processors" (1993), and
 * by the paper's methods B2 and B3 (Section 3, see nrng_b2 and nrng_b3), P2
 * (Section 4, see nrng_polar2) and Algorithm R (Section 5, see nrng_ratio):
 *
 *   Algorithm B1 (Box-Muller):  r = sigma sqrt(-2 ln(1 - u)),
 *                               x = r sin(2 pi v) + mu,  y = r cos(2 pi v) + mu;
 *   Algorithm P (Polar method): x, y uniform on [-1, 1), s = x^2 + y^2,
 *                               reject if s >= 1, else r = sigma sqrt(-2 ln(s)/s)
 *                               and return r x + mu, r y + mu.
 *
 * Uniform stream (identical in every entry point): counter c_i = seed +
 * offset + i (mod 2^64) and hash k_i = SplitMix64(c_i), one generator step
 * (add 0x9E3779B97F4A7C15, then the variant-13 mixer).
 *   - B1 pair k uses u = (k_{2k} >> 11) 2^-53 and v = (k_{2k+1} >> 11) 2^-53
 *     (u may be 0 but never 1, the paper's assumption in Section 2, note a).
 *     Output 2k is the sine value x, output 2k+1 the cosine value y.
 *   - Polar candidate j uses X = (int32)(k_{2j} >> 32) and
 *     Y = (int32)(k_{2j+1} >> 32), i.e. x = X 2^-31, y = Y 2^-31 in [-1, 1).
 *     With S = X^2 + Y^2 computed exactly in 64-bit integers, the candidate
 *     is accepted iff 0 < S < 2^62 (s < 1 decided exactly; s = 0 rejected to
 *     avoid the division by zero of step 4).  Accepted candidates are emitted
 *     in increasing j (stable order): the a-th accepted pair writes outputs
 *     2a and 2a+1.
 *   - If n is odd the last pair contributes only its first value.
 *   - Offsets and "consumed" counts are in uniforms (counter values), for both
 *     methods: B1 consumes 2 ceil(n/2); Polar consumes 2 (j_last + 1) where
 *     j_last is the candidate that supplied the last value.  Calling again with
 *     offset + consumed continues the same stream exactly.
 *
 * Precision: NRNG_F64 output is computed in FP64 throughout (the plain FP64
 * kernels).  NRNG_F32, NRNG_BF16 and NRNG_F16 are computed in FP32 (the Polar
 * kernel switches to FP64 for ln(s)/s when s < 2^-20, and Algorithm R takes
 * its acceptance decision in FP64 wherever FP32 cannot settle it) and rounded
 * to nearest even once into the output format.
 *
 * Conventions for every entry point:
 *   - Pointers named out and d_* are device pointers on the current HIP
 *     device, allocated and owned by the caller; the library never frees or
 *     retains them.  `out` may have any element alignment.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream);
 *     all work is enqueued asynchronously on it.  No entry point synchronises
 *     the device unless its comment says so.
 *   - Return value: NRNG_OK (0) or a negative nrng_status.  Argument errors
 *     are reported before anything is launched and nothing is written.
 *     Nothing prints and nothing aborts.
 *   - Sizes: n <= 2^62 for the Box-Muller family (B1, B2, B3); n <= 2^41 for
 *     the rejection methods (Polar, P2, R) and out_len <= 2^41 for a batch
 *     (their workspace holds one mask bit per candidate).  Larger sizes
 *     return NRNG_ERANGE before any launch.
 *   - The library keeps a per-device workspace (accept masks of the rejection
 *     methods, about one bit per candidate, tile prefix counts, batched tile
 *     tables).  Calls that use it (Polar, P2, R, batched) must be ordered on
 *     one stream per device; concurrent such calls on different streams of
 *     one device race.  The workspace grows on demand, which allocates; during
 *     stream capture growth is refused with NRNG_ECAPTURE, so call
 *     nrng_reserve() before capturing.
 */
#ifndef NRNG_H
#define NRNG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Output element types. */
enum nrng_dtype { NRNG_F64 = 0, NRNG_F32 = 1, NRNG_BF16 = 2, NRNG_F16 = 3 };

/* Methods for nrng_batched. */
enum nrng_method {
    NRNG_METHOD_B1 = 0,
    NRNG_METHOD_POLAR = 1,
    NRNG_METHOD_P2 = 2,
    NRNG_METHOD_B3 = 3,
    NRNG_METHOD_R = 4,
    NRNG_METHOD_B2 = 5
};

/* Status codes. */
enum nrng_status {
    NRNG_OK = 0,
    NRNG_EINVAL = -1,   /* bad pointer, non-finite mu/sigma, sigma < 0, bad method */
    NRNG_EDTYPE = -2,   /* unknown dtype */
    NRNG_ERANGE = -3,   /* size too large (counter range or workspace limits) */
    NRNG_EHIP = -4,     /* a HIP runtime call or kernel launch failed */
    NRNG_ENODEV = -5,   /* no usable GPU */
    NRNG_ECAPTURE = -6, /* the call would allocate while the stream is capturing */
    NRNG_ENOMEM = -7    /* device allocation failed */
};

/* Static description of a status code (never NULL). */
const char *nrng_strerror(int status);

/* Library version, major * 10000 + minor * 100 + patch. */
int nrng_version(void);

/* Initialise the current device: query it and allocate the base workspace.
 * Optional (every entry point initialises lazily); allocates, so not for use
 * during stream capture.  NRNG_ENODEV if no HIP device is usable. */
int nrng_init(void);

/* Pre-size the current device's workspace so that later calls with at most
 * max_n normals per single-stream Polar call, and batched calls with at most
 * max_streams streams and max_n normals in total, do not allocate (needed
 * before capturing such calls in a graph).  Allocates; not capturable. */
int nrng_reserve(uint64_t max_n, uint32_t max_streams);

/* ------------------------------------------------------------------------
 * Algorithm B1 (Box-Muller), Section 2, over one stream.
 *   seed, offset  the stream and the first counter used (uniform units)
 *   n             normals to write (0 is a no-op returning NRNG_OK)
 *   mu, sigma     mean and standard deviation (finite, sigma >= 0)
 *   out           n elements of `dtype`
 * Consumes exactly 2 ceil(n/2) uniforms.  Embarrassingly parallel: each pair
 * is computed independently and stored with 16-byte vector stores.
 * ---------------------------------------------------------------------- */
int nrng_boxmuller(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, void *out,
                   int dtype, void *stream);

/* ------------------------------------------------------------------------
 * Method B3 (Section 3), over one stream: Box-Muller with the square root
 * avoided by drawing two uniforms.  Pair k uses the uniforms u1, u2, u3 of
 * counters 3k, 3k + 1, 3k + 2 (same uniform definition as B1):
 *   m = max(u1, u2), u = m^2 (uniform on [0, 1), sqrt(u) = m);
 *   r = sigma m h(v) with v = (6u - 4)/(4 - 3u) for u <= 8/9 (h: the
 *   polynomial of nrng_polar2, degree 15 in FP64, 9 in FP32), else
 *   r = sigma sqrt(-ln(1 - u));
 *   t = 2 pi u3 - pi; output 2k = mu + cos(t) r sqrt(2), output 2k+1 =
 *   mu + sin(t) r sqrt(2) (written only if 2k+1 < n).
 * Consumes exactly 3 ceil(n/2) uniforms.  Arguments, errors and launch
 * configuration (nrng_tune_set kernel 0) as nrng_boxmuller. */
int nrng_b3(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, void *out, int dtype,
            void *stream);

/* ------------------------------------------------------------------------
 * Method B2 (Section 3), over one stream: B1 with the sine and cosine
 * computed inline.  Pair k uses the u and v of B1's pair k:
 *   r = sigma sqrt(-2 ln(1 - u));  y = (2 pi v - pi)/16 (|y| <= pi/16);
 *   sin y ~= s1 y + s3 y^3 + s5 y^5 + s7 y^7, cos y ~= c0 + c2 y^2 + c4 y^4 +
 *   c6 y^6 (the Chebyshev series of sin(y)/y and cos y in y^2 on
 *   [0, (pi/16)^2], truncated after T_3), then four doublings
 *   sin 2y = 2 sin y cos y, cos 2y = 1 - 2 sin^2 y;
 *   output 2k = r sin(16y) + mu, output 2k+1 = r cos(16y) + mu.
 * Since 16y = 2 pi v - pi, pair k equals B1's pair k negated about mu, up to
 * the approximation (absolute error below 2e-12 r in FP64).  The FP64 kernel
 * keeps the method's order of operations; the FP32 kernel reduces the angle
 * to a quarter turn first and its sine and cosine are accurate to about
 * 2^-20 absolute.  Consumes exactly 2 ceil(n/2) uniforms.  Arguments,
 * errors and launch configuration (nrng_tune_set kernel 0) as
 * nrng_boxmuller. */
int nrng_b2(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, void *out, int dtype,
            void *stream);

/* ------------------------------------------------------------------------
 * Algorithm P (Polar method), Section 2, over one stream.
 *   Arguments as nrng_boxmuller.  The acceptance test of step 3 and the
 *   compaction of accepted pairs (the paper's vector gather, Section 2, and
 *   the compress of triples (x_j, y_j, s_j), Section 4) run as three kernels
 *   on `stream`: a mask pass (hash, exact test, wavefront ballots -> one
 *   accept bit per candidate and a count per tile of candidates), a prefix
 *   scan of the tile counts, and a generate pass in which each lane takes
 *   consecutive accepted candidates, so accept masks and output indices are
 *   exact integers and only accepted candidates are transformed.  The
 *   candidate budget of the mask pass is the expected count plus four
 *   standard deviations; a stream that needs more continues exactly past it.
 *   d_consumed  optional device pointer (may be NULL): receives the number
 *               of uniforms consumed, 2 (j_last + 1).  Written
 *               asynchronously; no synchronisation.
 * ---------------------------------------------------------------------- */
int nrng_polar(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, void *out,
               int dtype, void *stream, uint64_t *d_consumed);

/* ------------------------------------------------------------------------
 * Method P2 (Section 4), over one stream: the Polar method with step 4
 * taking -ln(1 - s) in place of -ln(s) (1 - s is also uniform and
 * independent of the angle of (x, y)), so the radius factor is
 * sigma sqrt(2) g(s) with g(s) = sqrt(-ln(1 - s) / s), the function of
 * method B3 (Section 3).  For s <= 8/9, g is a polynomial in
 * v = (6 s - 4) / (4 - 3 s) (the Section 3 change of variable with rho = 1),
 * the truncated Chebyshev series of degree 15 in FP64 and degree 9 in FP32
 * (truncation errors 1.5e-11 and 6e-8); for s > 8/9, logarithm and square
 * root.  Outputs x r sqrt(2) + mu and y r sqrt(2) + mu.
 *   Candidates, pairing, stable order, odd-n rule, offsets and the consumed
 *   count are those of nrng_polar, except that step 3 rejects only s >= 1:
 *   the candidate (0, 0) (s = 0, g(0) = 1) is accepted and gives (mu, mu).
 *   The values differ from nrng_polar's (a different transform of the same
 *   candidates).  Same arguments, errors and workspace as nrng_polar; the
 *   launch configuration is the Polar one (nrng_tune_set kernel 1). */
int nrng_polar2(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, void *out,
                int dtype, void *stream, uint64_t *d_consumed);

/* ------------------------------------------------------------------------
 * Algorithm R (Section 5), the ratio method of Kinderman and Monahan in its
 * basic form, over one stream.  Candidate j uses the uniforms u = u_{2j} and
 * v = u_{2j+1} (same uniform definition as B1):
 *   x = sqrt(8/e) (v - 1/2) / (1 - u); accepted iff x^2 <= -4 ln(1 - u);
 *   the a-th accepted candidate writes output a = sigma x + mu.
 * (The test is the ratio method's, which gives the 8/sqrt(pi e) = 2.74
 * uniforms per normal that Section 5 states; the inequality as printed there
 * would accept 76% of candidates and not give a normal variable.)  Every
 * decision equals the FP64 evaluation of the test: an FP32 screen decides
 * where the two sides differ by more than 16 times its error bound, the FP64
 * test inside that thin band (under 1e-4 of candidates).  So accept masks,
 * output indices and consumed counts are exact; values are computed in the
 * output's precision class as for the other methods.  Runs as the Polar
 * kernels (mask, scan, generate) with one output per accepted candidate.
 * consumed = 2 (j_last + 1).  Arguments, errors, workspace and launch
 * configuration (nrng_tune_set kernel 1) as nrng_polar. */
int nrng_ratio(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, void *out, int dtype,
               void *stream, uint64_t *d_consumed);

/* Polar method with a device-resident counter offset, for repeated fills
 * captured in a HIP graph.  Section 4 notes that a compressing Polar
 * routine cannot tell in advance how many normals one vector of candidates
 * yields, and hides this behind a level of buffering (its user routine
 * RANN3 around the vector kernel RANN3B).  Here the stream position is kept
 * instead: the call reads the offset from *d_cursor when the kernel runs
 * and advances *d_cursor by the number of uniforms consumed, so that
 * successive calls (or graph replays) continue one stream and each yields
 * exactly n normals.  Launches the same three kernels as nrng_polar and
 * allocates nothing once the workspace is reserved (nrng_reserve(n, 0));
 * NRNG_ECAPTURE otherwise while capturing. */
int nrng_polar_dev(uint64_t seed, uint64_t *d_cursor, uint64_t n, double mu, double sigma, void *out,
                   int dtype, void *stream);

/* Algorithm P over one stream without any allocation, for callers that
 * cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, results
 * (bit for bit), consumed count and launch configuration as nrng_polar, but
 * the Polar kernels take their workspace from a fixed scratch array of
 * 8 MiB in device memory (one per device, held until the process ends)
 * instead of the library's growable workspace, so the call never calls
 * hipMalloc or hipFree, on its first call included.
 *   n  at most 2^26 (67,108,864) normals; larger n returns NRNG_ERANGE
 *      before anything is launched.
 * The scratch keeps the last call's contents and needs no clearing (every
 * kernel writes what the next one reads).  All calls of this entry point on
 * one device share that device's scratch: calls that overlap on one device
 * (on different streams, or from different host threads without ordering)
 * race and must not be made. */
int nrng_polar_noalloc(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, void *out,
                       int dtype, void *stream, uint64_t *d_consumed);

/* ------------------------------------------------------------------------
 * Many independent streams in one launch sequence.  Each stream is one call
 * of a single-stream method (B1 or P of Section 2, B2 or B3 of Section 3,
 * P2 of Section 4, R of Section 5); the paper's timings assume long vectors
 * (Section 3: many numbers generated per call), and serving thousands of
 * short, uneven streams in one launch recovers that on the GPU.  One small
 * set-up kernel builds the tile table on the device, then one persistent
 * kernel of the Box-Muller family, or the three Polar kernels, cover every
 * stream.
 *   method       NRNG_METHOD_B1, NRNG_METHOD_POLAR, NRNG_METHOD_P2, NRNG_METHOD_B3, NRNG_METHOD_R or
 *                NRNG_METHOD_B2
 *   nstreams     number of streams (0 is a no-op)
 *   d_seed[j], d_offset[j], d_n[j]  stream j's seed, first counter, length
 *   d_out_off[j] element offset of stream j's output in `out`; NULL means
 *                packed (exclusive prefix sum of d_n)
 *   d_mu[j], d_sigma[j]             per-stream mean and standard deviation
 *   out, out_len output buffer and its length in elements; a stream whose
 *                range [out_off, out_off + n) does not lie in [0, out_len)
 *                is skipped (invalid)
 *   d_consumed   optional (may be NULL): d_consumed[j] receives stream j's
 *                consumed uniforms, or UINT64_MAX if the stream was skipped.
 * Stream j's values equal those of nrng_boxmuller / nrng_polar / nrng_polar2 /
 * nrng_b3 / nrng_ratio / nrng_b2 called alone with (d_seed[j], d_offset[j],
 * d_n[j], d_mu[j], d_sigma[j]), bit for bit.
 * The set-up kernel fails the whole call on the device (every d_consumed[j]
 * = UINT64_MAX, nothing written) when the lengths of the valid streams total
 * more than out_len (possible only with explicit, overlapping d_out_off), or
 * when the tile table outgrows the workspace sized for out_len.  Valid
 * streams with overlapping ranges that pass this check are written in an
 * unspecified order.  Per-stream mu and sigma are not validated on the
 * host. */
int nrng_batched(int method, uint32_t nstreams, const uint64_t *d_seed, const uint64_t *d_offset,
                 const uint64_t *d_n, const uint64_t *d_out_off, const double *d_mu, const double *d_sigma,
                 void *out, uint64_t out_len, int dtype, void *stream, uint64_t *d_consumed);

/* The two halves of nrng_batched, for callers that refill the same set of
 * streams repeatedly or time the main kernel on its own.
 * nrng_batched_plan builds the tile table of the batch in the device
 * workspace (one small kernel; d_consumed as in nrng_batched, written for
 * skipped and empty streams and for every B1 stream); nrng_batched_exec runs
 * the persistent kernel over the most recent plan of the method's family on
 * this device (families below).  exec returns NRNG_EINVAL unless that plan
 * was made for the same method, dtype, launch variant, stream count and
 * layout (packed or not); d_n and d_out_off must hold the values the plan
 * saw.  A plan stays valid until the next plan or batched call of its
 * family on the device.  nrng_batched(...) is plan + exec.
 * nrng_batched_exec_part runs one half of exec's launch sequence, for timing
 * and profiling the kernels separately: part 1 = the Polar (or P2) mask and
 * scan kernels (nothing for B1 and B3), part 2 = the generate kernel (the B1 or B3
 * kernel for B1), part 0 = both (identical to nrng_batched_exec).  Part 2
 * reads what part 1 of the same plan left in the workspace, so it must
 * follow it (on the same stream, or ordered after it by an event) with no
 * other Polar call in between.  Same arguments and errors as
 * nrng_batched_exec, plus NRNG_EINVAL for a part outside 0..2.
 *
 * The two method families keep separate tables: the Box-Muller family (B1,
 * B3, B2) and the rejection family (Polar, P2, R; these also share the
 * candidate workspace).  A plan stays valid until the next plan or batched
 * call of its own family, so a batch of each family may be planned and run
 * at the same time on two streams; calls of one family must not overlap. */
int nrng_batched_plan(int method, uint32_t nstreams, const uint64_t *d_n, const uint64_t *d_out_off,
                      uint64_t out_len, int dtype, void *stream, uint64_t *d_consumed);
int nrng_batched_exec(int method, uint32_t nstreams, const uint64_t *d_seed, const uint64_t *d_offset,
                      const uint64_t *d_n, const uint64_t *d_out_off, const double *d_mu, const double *d_sigma,
                      void *out, int dtype, void *stream, uint64_t *d_consumed);
int nrng_batched_exec_part(int part, int method, uint32_t nstreams, const uint64_t *d_seed,
                           const uint64_t *d_offset, const uint64_t *d_n, const uint64_t *d_out_off,
                           const double *d_mu, const double *d_sigma, void *out, int dtype, void *stream,
                           uint64_t *d_consumed);

/* nrng_batched_exec_part with its main kernel timed: the same launches,
 * results and errors, except that the main kernel (the Box-Muller family's
 * batched kernel, or the Polar, P2 or R generate kernel) is dispatched with
 * hipExtLaunchKernel so that ev_start and ev_stop record that dispatch's own
 * start and end.  No marker is added to the stream, and
 * hipEventElapsedTime(ev_start, ev_stop) is the kernel's duration alone.
 *   part               0 (the whole exec) or 2 (the main kernel); part 1
 *                      has no main kernel (NRNG_EINVAL)
 *   ev_start, ev_stop  hipEvent_t handles created by the caller (with
 *                      timing enabled) on the stream's device; both are
 *                      required (NRNG_EINVAL if either is NULL).
 * The events are not recorded when nothing is launched (nstreams 0, or an
 * error return). */
int nrng_batched_exec_timed(int part, int method, uint32_t nstreams, const uint64_t *d_seed,
                            const uint64_t *d_offset, const uint64_t *d_n, const uint64_t *d_out_off,
                            const double *d_mu, const double *d_sigma, void *out, int dtype, void *stream,
                            uint64_t *d_consumed, void *ev_start, void *ev_stop);

/* ------------------------------------------------------------------------
 * Repeated fills through a HIP graph: capture one nrng_polar_dev launch
 * (with the workspace reserved beforehand) and return an instantiated graph
 * in *graph.  Each nrng_fillgraph_launch replays it on `stream`, refilling
 * `out` with the next n normals of the stream and advancing *d_cursor.
 * The capture uses `stream`, which must not be capturing already. */
int nrng_fillgraph_create(uint64_t seed, uint64_t *d_cursor, uint64_t n, double mu, double sigma, void *out,
                          int dtype, void *stream, void **graph);
int nrng_fillgraph_launch(void *graph, void *stream);
int nrng_fillgraph_destroy(void *graph);

/* ------------------------------------------------------------------------
 * Launch configuration.  kernel: 0 = B1 and B3 single stream, 1 = Polar, P2
 * and Algorithm R (single, device cursor and batched), 2 = B1 and B3
 * batched.  Sets the workgroup size and
 * per-thread unroll used for `dtype`; NRNG_EINVAL if that pair is not one of
 * the compiled variants (nrng_tune_variants lists them as (wg, unroll)
 * pairs).  grid_per_cu (0 = from the occupancy query) caps the persistent
 * grid at that many workgroups per compute unit. */
int nrng_tune_set(int kernel, int dtype, uint32_t wg, uint32_t unroll, uint32_t grid_per_cu);
int nrng_tune_get(int kernel, int dtype, uint32_t *wg, uint32_t *unroll, uint32_t *grid_per_cu);
int nrng_tune_variants(int kernel, uint32_t *pairs, int max_pairs);

/* Load a launch-configuration table (as written by the autotuner) from a text
 * file: one entry per line, "<kernel> <dtype> <wg> <unroll> <grid_per_cu>",
 * kernel one of b1, polar, b1_batched (kernels 0, 1, 2 above), dtype one of
 * f64, f32, bf16, f16; '#' starts a comment.  All entries are checked first
 * (names, and (wg, unroll) a compiled variant) and then applied together;
 * NRNG_EINVAL for a NULL or unreadable path or any bad entry, in which case
 * nothing is changed.  Entries not in the file keep their values. */
int nrng_tune_load(const char *path);

/* ------------------------------------------------------------------------
 * Test hooks: the production per-pair arithmetic and compaction fed from
 * explicit inputs instead of the hash stream.
 *
 * nrng_test_b1_words: pair p uses u-word d_words[2p] and v-word
 *   d_words[2p+1] (64-bit hash words); writes out[2p], out[2p+1].
 * nrng_test_b3_words: the same for method B3, three words per pair (u1,
 *   u2, u3), d_words holding 3 npairs words.
 * nrng_test_b2_words: the same as nrng_test_b1_words for method B2.
 * nrng_test_polar_xy: candidate j is (d_xy[2j], d_xy[2j+1]); accepted
 *   candidates are written compactly in order to out (capacity 2 ncand);
 *   d_mask_words (ceil(ncand/64) words, bit j%64 of word j/64 = accept) and
 *   *d_count (number accepted) are written.
 * nrng_test_polar2_xy: the same for method P2 (accepts 0 <= S < 2^62).
 * nrng_test_ratio_words: Algorithm R on explicit candidates, candidate j
 *   being the 64-bit words (d_words[2j], d_words[2j+1]) read as u and v;
 *   outputs, masks and count as nrng_test_polar_xy (one output per accepted
 *   candidate).
 * nrng_ratio_trace: Algorithm R's accept masks and word prefixes over
 *   candidates [0, ncand) of stream (seed, offset), as nrng_polar_trace.
 * nrng_polar_trace: the accept masks and, per 64-candidate word, the output
 *   pair index of its first candidate (exclusive prefix), for candidates
 *   [0, ncand) of stream (seed, offset), produced by the production Polar
 *   mask pass (predicate and ballots) and prefix scan.
 * nrng_test_polar_budget: nrng_polar with the candidate budget forced to
 *   `words` (>= 1) words of 64 candidates, to exercise the exact
 *   continuation path that runs when a stream needs more candidates than its
 *   budget.  nrng_test_ratio_budget: the same for nrng_ratio.
 * ---------------------------------------------------------------------- */
int nrng_test_b1_words(const uint64_t *d_words, uint64_t npairs, double mu, double sigma, void *out, int dtype,
                       void *stream);
int nrng_test_b3_words(const uint64_t *d_words, uint64_t npairs, double mu, double sigma, void *out, int dtype,
                       void *stream);
int nrng_test_b2_words(const uint64_t *d_words, uint64_t npairs, double mu, double sigma, void *out, int dtype,
                       void *stream);
int nrng_test_polar_xy(const int32_t *d_xy, uint64_t ncand, double mu, double sigma, void *out, int dtype,
                       uint64_t *d_mask_words, uint64_t *d_count, void *stream);
int nrng_test_polar2_xy(const int32_t *d_xy, uint64_t ncand, double mu, double sigma, void *out, int dtype,
                        uint64_t *d_mask_words, uint64_t *d_count, void *stream);
int nrng_test_ratio_words(const uint64_t *d_words, uint64_t ncand, double mu, double sigma, void *out, int dtype,
                          uint64_t *d_mask_words, uint64_t *d_count, void *stream);
int nrng_ratio_trace(uint64_t seed, uint64_t offset, uint64_t ncand, uint64_t *d_mask_words,
                     uint64_t *d_word_prefix, void *stream);
int nrng_polar_trace(uint64_t seed, uint64_t offset, uint64_t ncand, uint64_t *d_mask_words,
                     uint64_t *d_word_prefix, void *stream);
int nrng_test_polar_budget(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, void *out,
                           int dtype, uint32_t words, void *stream, uint64_t *d_consumed);
int nrng_test_ratio_budget(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, void *out,
                           int dtype, uint32_t words, void *stream, uint64_t *d_consumed);

/* ------------------------------------------------------------------------
 * Measurement probes (roofline ceilings and counter calibration).
 * nrng_probe_store: write nbytes (multiple of 16) of a fixed pattern with
 *   16-byte stores -- the store-only HBM ceiling.
 * nrng_probe_copy: copy nbytes (multiple of 16) from src to dst -- a kernel
 *   of known traffic for scaling hardware byte counters.
 * nrng_probe_hash: nhash SplitMix64 hashes of counters seed + i, xor-reduced
 *   into d_sink[0..gridsize) -- the hash-only VALU ceiling.
 * ---------------------------------------------------------------------- */
int nrng_probe_store(void *out, uint64_t nbytes, void *stream);
/* nrng_probe_store_variant: the store-only ceiling in a chosen form:
 *   nontemporal != 0 writes with nontemporal 16-byte stores
 *   (global_store_dwordx4 ... nt), else plain ones; blocks_per_cu
 *   workgroups of 256 threads per compute unit (1 to 32); unroll 16-byte
 *   stores per thread per step (1, 2, 4 or 8), each wave store writing
 *   1 KiB contiguously.  NRNG_EINVAL for other values or nbytes not a
 *   multiple of 16. */
int nrng_probe_store_variant(void *out, uint64_t nbytes, int nontemporal, uint32_t blocks_per_cu, uint32_t unroll,
                             void *stream);
int nrng_probe_copy(void *dst, const void *src, uint64_t nbytes, void *stream);
int nrng_probe_hash(uint64_t seed, uint64_t nhash, uint64_t *d_sink, uint64_t sink_len, void *stream);

/* Issue-rate probe, for the cost model of the ALU roofline: (device CUs x 8)
 * workgroups of 256 lanes each run 8 independent chains of `iters`
 * repetitions of one VALU instruction, then write the xor of their chains to
 * d_sink[g] (32-bit words, only for g < sink_len).  op selects the
 * instruction: 0 v_add_u32, 1 v_mul_lo_u32, 2 v_mul_hi_u32, 3 v_mul_u32_u24,
 * 4 v_fma_f32, 5 v_cvt_f32_u32, 6 v_log_f32, 7 v_sin_f32, 8 v_sqrt_f32,
 * 9 v_rcp_f32, 10 v_lshrrev_b64, 11 v_lshl_add_u64, 12 v_mad_u64_u32,
 * 13 v_mad_i64_i32, 14 v_fma_f64.  Lane operations per launch:
 * CUs x 8 x 256 x 8 x iters.  NRNG_EINVAL for another op, a NULL sink or
 * sink_len 0. */
int nrng_probe_valu(int op, uint32_t iters, uint32_t *d_sink, uint64_t sink_len, void *stream);

/* Number of compute units of the current device (0 if none). */
int nrng_device_cus(void);

#ifdef __cplusplus
}
#endif

#endif /* NRNG_H */
