/* Exact 2D least-median-of-squares (LMS) line fitting on AMD Instinct MI355X
 * (gfx950). C ABI.
 *
 * Method: Shapira & Hassner, "GPU-Based Computation of 2D Least Median of
 * Squares with Applications to Fast and Robust Line Detection", arXiv
 * 1510.01041.
 *   - Section 1, Eq. (1): the LMS line y = theta1*x + theta2 minimises the
 *     median of the squared residuals r_k = y_k - theta1*x_k - theta2.
 *   - Section 3.1: equivalently, the thinnest vertical slab holding h points;
 *     the line bisects it.
 *   - Sections 3.2-3.4 and Algorithm 1: the optimal slope is the slope of a
 *     pair of points (a vertex of the dual line arrangement), so an exhaustive
 *     search over all n(n-1)/2 pair slopes is exact.
 *
 * Conventions shared by every entry point:
 *   - Points are n interleaved FP64 pairs (x0, y0, x1, y1, ...), in DEVICE
 *     memory unless the name says "host". The caller owns every input and
 *     output buffer. The library owns only a workspace per (device, stream),
 *     which it grows on demand and releases in lms_shutdown().
 *   - h is the number of points the slab must hold; h = 0 selects the low
 *     median floor(n/2) + 1. Valid range: 2 <= h <= n.
 *   - Supported sizes: 2 <= n <= LMS_MAX_N.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). All
 *     device work is enqueued on it. The call returns once the work is
 *     enqueued; the results are valid after the stream is synchronised.
 *   - Argument errors are detected on the host before anything is enqueued,
 *     and return a negative status; lms_last_error() then holds a message.
 *     Data-dependent conditions (non-finite input, all x equal) are detected
 *     on the device and reported in the result's `status` field.
 *   - Calls on different streams may run concurrently. Calls on one stream are
 *     ordered. The library is thread-safe.
 */
#ifndef LMS_H
#define LMS_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LMS_MAX_N 16384

typedef enum {
  LMS_OK = 0,
  LMS_OK_DEGENERATE = 1,  /* all x equal: no pair has a finite slope; theta1 := 0 */
  LMS_ERR_ARG = -1,       /* bad argument (host check) */
  LMS_ERR_NONFINITE = -2, /* a coordinate is NaN or infinite (device check) */
  LMS_ERR_DEVICE = -3,    /* a HIP call failed */
  LMS_ERR_NOMEM = -4,     /* workspace allocation failed */
  LMS_ERR_CAPACITY = -5   /* lms_solve under a max_workspace limit: more screen
                             survivors than the limited list holds. (No seed error
                             exists: any seed slope, even NaN, is only a bound.) */
} lms_status;

/* Result of one solve. 128 bytes, written to device memory by lms_solve.
 * On a negative status the FP64 fields are NaN. */
typedef struct lms_result {
  double theta1;     /* slope of the LMS line (a pair slope; 0 if degenerate) */
  double theta2;     /* intercept: midpoint of the narrowest window */
  double half_width; /* w = (z_hi - z_lo)/2; the LMS criterion is w*w */
  double width;      /* z_hi - z_lo: vertical height of the thinnest slab */
  double z_lo, z_hi; /* window ends, z = fma(-theta1, x, y) */
  int32_t pair_i, pair_j; /* a pair (i < j) whose slope attains the result */
  int32_t status;         /* lms_status */
  int32_t h;              /* h actually used */
  uint64_t candidates;    /* non-vertical pairs, n(n-1)/2 - vertical */
  uint64_t vertical;      /* pairs with x_i == x_j, skipped */
  uint64_t survivors;     /* pairs the FP32 screen passed to the FP64 check */
  uint64_t point_evals;   /* FP32 residuals of the band test (FMA + one compare each) */
  uint64_t dir_evals;     /* FP32 residuals of the one-sided tests (FMA + four compares) */
  uint64_t band_pass;     /* pairs that passed the band test */
  uint64_t bin_pass;      /* pairs the slope-bin screen passed to the FP32 test
                             (lms_solve; 0 where that screen did not run) */
  uint64_t bins;          /* slope bins per anchor of that screen (0: not run;
                             2048: the pruned screen of the slope range ran) */
} lms_result;

/* Flags for lms_options.flags */
#define LMS_F_GRAPH 2u    /* lms_solve and lms_solve_batched: capture the pipeline in a
                             hipGraph on the first call and replay it on later calls
                             with the same pointers, problem shape, options and
                             stream (the input values may change). The graph owns a
                             workspace until lms_shutdown. */
#define LMS_F_NO_PRUNE 1u /* no width bound: the screen keeps every pair whose anchored
                             window can hold h points at all (slow; for tests) */
#define LMS_F_RANGE 4u    /* lms_solve: bound the optimal slope by exact windows at a
                             grid of slopes (two grids) and run the slope-bin screen
                             on the anchors and points that range leaves, at any n
                             (by default above 4096 points; the second grid above
                             8192) */
#define LMS_F_NO_RANGE 8u /* lms_solve: never (LMS_F_RANGE wins over it) */

typedef struct lms_options {
  uint32_t struct_size; /* sizeof(lms_options) */
  uint32_t flags;       /* LMS_F_* */
  int32_t seed_pairs;   /* random pair slopes evaluated exactly before the screen
                           to set the initial width bound; -1 = automatic (the tuned
                           value, else 127 for lms_solve and 31 per problem for
                           lms_solve_batched) */
  int32_t tile_regs;    /* 0 = automatic (tuned, else all points in registers up to
                           4096). Otherwise the number of 64-point chunks of the
                           screen kept in registers (1, 16, 32 or 64); the other
                           points stream from LDS. */
  const double* d_seed_theta; /* optional device array of extra seed slopes (any
                                 real values; they only tighten the initial bound) */
  int64_t n_seed_theta;       /* length of d_seed_theta */
  int32_t tile_batches; /* 0 = automatic; otherwise 64-partner batches per work item
                           of the screen (1..64) */
  int32_t window_pairs; /* lms_solve with device seed slopes: 0, or the number of
                           pairs (<= 65536) drawn among the points of the narrowest
                           seed slope's window and evaluated exactly as further
                           seeds; a second round draws as many from the narrowest
                           window of the first round's pairs. A slope near the LMS
                           line puts mostly inliers in its window, so these pairs
                           give a tight bound. Ignored by lms_solve_batched. */
  int32_t bins_log2;    /* lms_solve: slope bins per anchor of the first screen,
                           2^bins_log2 plus one per thread of its workgroup
                           (11..15; raised to at least 2n); 0 = automatic
                           (tuned, else about 2n); -1 = no slope-bin screen (every
                           pair goes through the FP32 test) */
  int32_t reserved;
  uint64_t max_workspace; /* 0 = no limit. Otherwise the most device memory, in bytes,
                           that the call's own workspace may take: lms_solve shrinks
                           the survivor list to 65536 slots, then the slope-bin pass
                           list (an overflowing list makes the exhaustive FP32
                           screen run instead, same result), then the survivor list
                           again (more survivors than it holds give
                           LMS_ERR_CAPACITY), each to at least 1024 slots;
                           lms_solve_batched shrinks its pass and survivor lists
                           and re-solves the problems whose survivors did not fit
                           (see there). If even the fixed part does not fit:
                           LMS_ERR_NOMEM. Read only when struct_size covers it. */
  const float* d_net_params; /* lms_solve: device, LMS_NET_PARAMS FP32 seed-network
                           parameters, or NULL. When set, the solve first runs the
                           network on the points (lms_net_infer, max_points 2048)
                           and uses its slope as the device seed slope (exclusive
                           with d_seed_theta; window_pairs applies to it). The
                           result stays exact whatever the network predicts. Read
                           only when struct_size covers it. */
} lms_options;

/* Tile choice found by the autotuner for one size class. */
typedef struct lms_tuning {
  int32_t tile_regs, tile_batches, seed_pairs, bins_log2;
  double ms;     /* median time of one solve (or one batched pass) with this choice */
  int32_t range; /* lms_solve's slope range: 0 automatic, 1 always, -1 never */
  int32_t reserved;
} lms_tuning;

/* Exact LMS line of one point set (Eq. (1); Algorithm 1's exhaustive search
 * over pair slopes).
 * d_xy: device, n x 2 FP64 interleaved. d_out: device, one lms_result.
 * opt may be NULL (defaults). The result is bit-identical to the FP64
 * reference search on the same input: the slab width, slope and window of the
 * canonical minimiser, ordered by (width, theta1, z_lo). */
lms_status lms_solve(const double* d_xy, int64_t n, int64_t h, lms_result* d_out,
                     const lms_options* opt, void* stream);

/* lms_solve without any allocation, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc). The workspace is one static device array of
 * LMS_NOALLOC_WORKSPACE bytes in the library, held by every GPU the library
 * runs on until the process ends; its device address is looked up once per
 * device. The solve's lists shrink to fit it as under opt->max_workspace
 * (an overflowing slope-bin list falls back to the exhaustive FP32 screen;
 * more survivors than the shrunk list holds give LMS_ERR_CAPACITY); a size
 * whose fixed part does not fit is rejected with LMS_ERR_ARG. LMS_F_GRAPH is
 * rejected (the caller may capture the stream itself). All calls on one GPU
 * share the array, and every call initialises the state it reads: calls that
 * overlap on one GPU race (serialise them, e.g. on one stream). Arguments and
 * results otherwise as lms_solve, bit for bit. */
#define LMS_NOALLOC_WORKSPACE (96u << 20)
lms_status lms_solve_noalloc(const double* d_xy, int64_t n, int64_t h, lms_result* d_out,
                             const lms_options* opt, void* stream);

/* Device bytes of the workspace lms_solve would use for (n, h, opt) (after
 * any max_workspace limit), into *bytes; LMS_ERR_ARG or LMS_ERR_NOMEM as
 * lms_solve would return them. Enqueues nothing. */
lms_status lms_workspace_size(int64_t n, int64_t h, const lms_options* opt, uint64_t* bytes);

/* Exact LMS lines of B independent point sets in one pass (Section 5 applies
 * one LMS per Hough peak; this is that many-small-problems form).
 * d_xy: device, all points, n_b x 2 FP64 interleaved per problem.
 * d_offsets: device, B+1 int64: problem b holds points [d_offsets[b],
 *   d_offsets[b+1]), each 2 <= n_b <= LMS_BATCH_MAX_N (a smaller problem gets
 *   status LMS_ERR_ARG in its own result; the others are solved).
 * h_offsets: the same offsets in host memory, or NULL (the library then copies
 *   them, which synchronises the stream). The work plan is built from them
 *   and cached per (pointers, stream, offsets).
 * d_h: device, B int32 values of h, or NULL for floor(n_b/2)+1 each.
 * d_out: device, B results. opt->seed_pairs is per problem (default 31).
 * With LMS_F_GRAPH the kernels are captured in a hipGraph on the first call
 * and replayed afterwards; the inputs may change between calls, the pointers
 * and offsets may not (otherwise the plan and graph are rebuilt).
 * Capacity: survivors of all problems share one list. When the batch has more
 * pairs than that list holds (by default above 2^24 pairs, or under
 * opt->max_workspace), the call waits for the batch once, and every problem
 * whose survivors did not fit is solved again by lms_solve (whose list holds
 * all pairs of a problem of this size) into its own result: every valid
 * problem gets its exact answer. Otherwise the call only enqueues.
 * Problems are limited to 2^30 points in all (d_offsets[B] <= 2^30). */
#define LMS_BATCH_MAX_N 4096
lms_status lms_solve_batched(const double* d_xy, const int64_t* d_offsets,
                             const int64_t* h_offsets, int64_t B, const int32_t* d_h,
                             lms_result* d_out, const lms_options* opt, void* stream);

/* Autotuner. Times lms_solve on the caller's point set (device memory) with
 * HIP events on `stream`, `reps` runs each (median), and keeps the fastest
 * choice for the size class next_pow2(n) of this device. It sweeps what moves
 * the time: the slope-bin screen's bins per anchor (every allowed 2^k), the
 * slope range (automatic, always, never), the random seed pairs (127, 63, 255),
 * then the FP32 screen's tiles (register chunks vs LDS streaming, partner
 * batches per work item). Every candidate must return the same line as the
 * defaults, bit for bit (LMS_ERR_DEVICE otherwise). Later lms_solve calls
 * with automatic options use the choice. If the environment variable
 * LMS_TUNE_FILE names a file, the table is read from it at the first use and
 * written back after each tuning. Synchronises the stream. */
lms_status lms_autotune(const double* d_xy, int64_t n, int64_t h, int32_t reps, void* stream,
                        lms_tuning* out);
/* Forgets every tuned choice of this process (solves use the defaults again;
 * a LMS_TUNE_FILE is not read again). */
void lms_tuning_clear(void);
/* The same for lms_solve_batched, on the caller's batch (the arguments are
 * those of lms_solve_batched), for the batch's size class (next_pow2 of its
 * largest problem): the random seed pairs per problem (15, 31, 63) times the
 * bins of the per-wavefront screen of problems up to 1024 points (2^12,
 * 2^11; out->bins_log2). A choice is kept only if every problem gets the
 * default settings' status and width bit for bit. */
lms_status lms_autotune_batched(const double* d_xy, const int64_t* d_offsets,
                                const int64_t* h_offsets, int64_t B, const int32_t* d_h,
                                lms_result* d_out, int32_t reps, void* stream, lms_tuning* out);

/* Synchronous convenience: host input, host output. Copies the points to the
 * device, solves on a library-owned stream and copies the result back. */
lms_status lms_solve_host(const double* xy, int64_t n, int64_t h, lms_result* out,
                          const lms_options* opt);

/* F(theta) at m given slopes: for each slope the narrowest window of h
 * consecutive values of z_k = fma(-theta, x_k, y_k) (the bracelet at that
 * dual u-coordinate, Section 3.2; Algorithm 1's per-vertex sort and window).
 * d_theta: device, m FP64. d_out: device, m x 3 FP64 (width, z_lo, z_hi);
 * among equally narrow windows the lowest. */
lms_status lms_eval_slopes(const double* d_xy, int64_t n, int64_t h, const double* d_theta,
                           int64_t m, double* d_out, void* stream);

/* Verdict of the FP32 screen for m given pairs against a width bound W (an
 * FP64 value that the optimal slab width is known not to exceed). For each
 * pair (d_pairs[2t], d_pairs[2t+1]), anchored on its first member, writes
 * d_verdict[t] = 1 if the screen
 * keeps the pair for the FP64 check, 0 if it proves that no anchored window of
 * width <= W exists at the pair's slope, 2 if the pair is vertical, -1 if an
 * index is outside [0, n).
 * Exposes the pruning test of lms_solve for soundness testing. */
lms_status lms_screen_pairs(const double* d_xy, int64_t n, int64_t h, double W,
                            const int32_t* d_pairs, int64_t m, int32_t* d_verdict,
                            void* stream);

/* Stage timing. Between lms_profile_begin() and lms_profile_end(), every
 * lms_solve records HIP events on its own stream around its six stages
 * (prep, seed evaluation, slope-bin screen, FP32 screen, FP64 recheck,
 * finalize); the events add no synchronisation. lms_profile_end() waits for
 * those events, writes the summed milliseconds per stage to
 * ms[0..LMS_NSTAGES) and returns the number of solves timed (negative status
 * on a HIP error). */
#define LMS_NSTAGES 6
void lms_profile_begin(void);
int64_t lms_profile_end(double* ms);

/* ---- Learned seed slope (a proposal for the initial width bound) ----
 * A small point-set network: per point 2 -> 64 -> 64 (ReLU), max-pool over
 * the points, head 64 -> 64 -> 2 (ReLU between), with BF16 weights (rounded
 * from FP32 masters) and FP32 accumulation. It predicts (cos 2phi, sin 2phi)
 * of the LMS line's angle phi in each set's normalised frame. Its slope only
 * seeds lms_solve through lms_options.d_seed_theta; since F(theta) >= the
 * optimum for every theta (Eq. (1)), the result stays exact for any
 * prediction. Parameters: LMS_NET_PARAMS FP32 values, packed
 * W1[64][2] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[2][64] b4[2].
 * Sets are CSR like lms_solve_batched (d_offsets, B+1 int64). */
#define LMS_NET_PARAMS 8642

/* Per set, per coordinate, a robust frame: the centre is the lower median
 * (rank floor((m-1)/2)) of a fixed sample of m points (all points up to 255,
 * else indices floor(k n / 255), k < 255), the scale the lower median of the
 * absolute deviations from it (the MAD), else the largest deviation, else 1;
 * up to half of the points being outliers moves neither. Writes d_pts (float2
 * per point, (p - centre) / scale) and d_scale (B x 4 FP64: cx, cy, sx, sy). */
lms_status lms_net_prepare(const double* d_xy, const int64_t* d_offsets, int64_t B, float* d_pts,
                           double* d_scale, void* stream);
/* Forward pass: d_out (B x 2 FP32) and, if d_g is not NULL, the pooled
 * features (B x 64 FP32) that lms_net_backward needs. */
lms_status lms_net_forward(const float* d_params, const float* d_pts, const int64_t* d_offsets,
                           int64_t B, float* d_out, float* d_g, void* stream);
/* Gradient of the mean over sets of 0.5 ||out - target||^2 (targets B x 2).
 * The max-pool routes each channel's gradient to the first point attaining
 * the maximum; the BF16 roundings pass gradients straight through.
 * d_grad_set: B x LMS_NET_PARAMS scratch; d_grad: LMS_NET_PARAMS, the sum
 * over sets in set order; d_loss: B per-set contributions to the mean loss. */
lms_status lms_net_backward(const float* d_params, const float* d_pts, const int64_t* d_offsets,
                            int64_t B, const float* d_target, const float* d_out,
                            const float* d_g, float* d_grad_set, float* d_grad, float* d_loss,
                            void* stream);
/* One bias-corrected Adam step (step >= 1) on the FP32 masters. */
lms_status lms_net_adam(float* d_params, float* d_m, float* d_v, const float* d_grad, int64_t step,
                        float lr, float beta1, float beta2, float eps, void* stream);
/* Inference for B sets, spread over many workgroups per set (the max-pool is
 * order-free, so the pooled features, outputs and slopes equal those of
 * lms_net_prepare + lms_net_forward + lms_net_slopes on the same points): the
 * frame of each set, then the features pooled over at most max_points points
 * of it (a set of n > max_points points is read at indices
 * floor(j n / max_points), j < max_points; the frame always comes from the
 * whole set), the head and the seed slope into d_theta (device, B FP64); the
 * raw outputs into d_out (device, B x 2 FP32) if not NULL. max_set bounds the
 * largest set (it sizes the grid). Scratch is a library workspace per stream. */
lms_status lms_net_infer(const float* d_params, const double* d_xy, const int64_t* d_offsets,
                         int64_t B, int64_t max_set, int32_t max_points, double* d_theta,
                         float* d_out, void* stream);
/* Seed slopes in the original frames: tan(atan2(out1, out0)/2) * sy / sx. */
lms_status lms_net_slopes(const float* d_out, const double* d_scale, int64_t B, double* d_theta,
                          void* stream);

/* ---- Algorithm 1 as stated (the ablation lms_solve is measured against) ----
 * Section 3.4, Algorithm 1, with the kernels of Section 3.6: every vertex of
 * the dual arrangement (pair slope) is materialised in an array; each vertex
 * gets one workgroup that computes all n intercepts z_k = fma(-theta, x_k,
 * y_k) at its slope, sorts them (bitonic, LDS, +inf padding to a power of
 * two) and reads the bracelet hanging from the vertex, h - 1 ranks away; a
 * min-reduction over the bracelet array gives the answer. The pair's own two
 * intercepts are set to exactly z_i, and the vertex occupies every rank
 * holding that value, r_lo..r_hi.
 *   LMS_RULE_TIED:    upward from r_lo or downward to r_hi, the shorter that
 *                     fits. The minimum is the LMS width (equioscillation puts
 *                     the optimal slab's edge through a vertex, Section 3.3).
 *   LMS_RULE_LITERAL: the printed far end X[(k + |P|/2) mod |P|] with
 *                     k = r_lo (up from k if it fits, else down to k): the rule
 *                     as printed, which leaves the tie open and can miss the
 *                     optimum.
 * d_xy: device, n x 2 FP64 interleaved, 2 <= n <= LMS_ALG1_MAX_N; h as for
 * lms_solve. d_out: device, one lms_result: the minimum bracelet by (length,
 * theta, lower end), then (i, j); survivors = candidates (every vertex is
 * sorted). Argument errors return LMS_ERR_ARG before anything is enqueued;
 * non-finite input gives status LMS_ERR_NONFINITE in the result; all x equal
 * gives LMS_OK_DEGENERATE with slope 0. Work O(n^3 log^2 n), workspace about
 * 48 n^2 / 2 bytes (library-owned, per stream). */
#define LMS_ALG1_MAX_N 2048
#define LMS_RULE_TIED 0
#define LMS_RULE_LITERAL 1
lms_status lms_solve_bracelets(const double* d_xy, int64_t n, int64_t h, int32_t rule,
                               lms_result* d_out, void* stream);

/* ---- Random sampling before the exact search (approximate) ----
 * Section 5: the LMS step of the line detector can be accelerated by randomly
 * sampling the feature points that voted for a Hough cell. Draws m of the n
 * points without replacement and returns the exact LMS line of the sample
 * (lms_solve on the sample, with `opt`); the line is an estimate of the whole
 * set's, not its exact LMS line. The sample is the m points with the smallest
 * keys mix64(seed + (k + 1) * 0x9E3779B97F4A7C15), the (k+1)-th SplitMix64
 * output for state `seed` (Steele, Lea and Flood, OOPSLA 2014), taken in index
 * order; equal keys go to the lower index.
 * d_xy: device, n x 2 FP64, 2 <= n <= LMS_SAMPLE_MAX_N. m: 2 <= m <= min(n,
 * LMS_MAX_N); m = n gives the exact solve. h: 0 for the sample's low median
 * floor(m/2) + 1, else the same fraction of the sample, ceil(h m / n) (at
 * least 2). d_out: device, one lms_result of the sample's solve (candidates
 * and vertical count the sample's pairs); pair_i and pair_j are indices into
 * d_xy. Argument errors return LMS_ERR_ARG before anything is enqueued. The
 * sample buffer is a library-owned workspace per stream. */
#define LMS_SAMPLE_MAX_N (1 << 30)
lms_status lms_solve_sampled(const double* d_xy, int64_t n, int64_t h, int64_t m, uint64_t seed,
                             lms_result* d_out, const lms_options* opt, void* stream);

/* ---- Line detection: coarse Hough transform, then LMS per peak ----
 * Section 5: a standard Hough transform with a coarse polar accumulator only
 * locates the feature points of each putative line; an exact LMS fit of the
 * points that voted for each accumulator peak then gives the line, so that up
 * to half of a cell's points may be noise or belong to another structure.
 *   - Accumulator: angle bins theta_b = b * d_theta (degrees, converted as
 *     b * (d_theta * pi/180)), b = 0 .. ceil(180 / d_theta) - 1, with cos and
 *     sin taken on the host (libm); rho = x cos theta_b + y sin theta_b in
 *     FP64 (two products and a sum), bin floor((rho + width - 1) / d_rho),
 *     floor((2 (width - 1) + height - 1) / d_rho) + 1 bins. Every pixel votes
 *     once per angle bin.
 *   - Peaks: cells with at least min_votes votes that are local maxima of
 *     their 3x3 neighbourhood (above the earlier neighbours in cell order, at
 *     least equal to the later ones); the max_lines strongest, by votes, then
 *     lower cell index.
 *   - Supporting set of a peak: the pixels that voted for it. Sets larger than
 *     max_support are sampled down to max_support points, the pixels with the
 *     smallest keys mix64(seed + (p + 1) * 0x9E3779B97F4A7C15) by pixel index
 *     p (the draw of lms_solve_sampled; the paper's random sampling of a
 *     cell's points). A steep line (normal within 45 degrees of the x axis,
 *     |cos theta_b| > |sin theta_b|) is fitted transposed, as x = theta1 y +
 *     theta2.
 *   - Fits: lms_solve_batched on all sets, h = floor(n/2) + 1.
 * d_pix: device, N x 2 int32 (x, y) pixel coordinates, 0 <= x < width,
 * 0 <= y < height (others vote nowhere). d_acc: optional device array of
 * n_theta x n_rho int32 that receives the accumulator (row = angle bin); NULL
 * keeps it in the library's workspace. lines: HOST array of max_lines; the
 * number of peaks found goes to *n_lines (host). Synchronous: it waits once
 * for the supporting-set sizes (the batched fit is planned from them) and
 * once for the fits. Argument errors return LMS_ERR_ARG. */
#define LMS_HOUGH_MAX_LINES 1024
typedef struct lms_hough_params {
  uint32_t struct_size;   /* sizeof(lms_hough_params) */
  int32_t width, height;  /* image size in pixels, 1 .. 2^20 */
  int32_t max_lines;      /* peaks to fit, 1 .. LMS_HOUGH_MAX_LINES */
  double d_rho;           /* rho bin width in pixels (>= 0.25) */
  double d_theta_deg;     /* angle bin width in degrees, (0, 180] */
  int32_t min_votes;      /* votes a peak needs (>= 2) */
  int32_t max_support;    /* largest set fitted, 2 .. LMS_BATCH_MAX_N */
  uint64_t seed;          /* seed of the sampling of larger sets */
} lms_hough_params;
typedef struct lms_line {
  int32_t theta_bin, rho_bin; /* the peak's cell */
  int32_t votes;              /* its votes (= the supporting pixels) */
  int32_t support, fitted;    /* supporting pixels; points fitted (after sampling) */
  int32_t transposed;         /* 1: result is the fit x = theta1 y + theta2 */
  int32_t reserved[2];
  lms_result result;          /* the LMS fit of the (transposed) set */
} lms_line;
lms_status lms_detect_lines(const int32_t* d_pix, int64_t N, const lms_hough_params* params,
                            int32_t* d_acc, lms_line* lines, int32_t* n_lines, void* stream);

const char* lms_status_str(int status);
/* Message for the last failing call on this thread ("" if none). */
const char* lms_last_error(void);
/* Frees every cached workspace. Call only when no work is in flight. */
void lms_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif
