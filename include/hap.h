/*
 * libhap -- Hierarchical Affinity Propagation (HAP) on AMD MI355X (gfx950).
 *
 * C ABI of the HIP library.  All pointers are plain addresses: "device" means
 * memory the HIP runtime allocated on the GPU the stream belongs to (for
 * example a torch tensor's data_ptr()), "host" means ordinary CPU memory.
 * No call takes ownership of caller memory.
 *
 * Problem statement (Section 2 and Algorithm 1 of Rose et al., "Parallel
 * Hierarchical Affinity Propagation with MapReduce", arXiv 1403.7394): the
 * input is a dense N x N similarity S with s_ij <= 0 whose diagonal holds the
 * preferences, a number of levels L and a damping factor lambda; the method
 * iterates the responsibility / availability updates (Eq. 2.1-2.3) and the
 * inter-level messages tau, phi and the cluster preference c (Eq. 2.4-2.6) at
 * every level, and outputs the exemplar e^l_i = argmax_j (alpha^l_ij + rho^l_ij)
 * of every point at every level (Eq. 2.8).
 *
 * Layout: matrices are row-major with a leading dimension (elements between the
 * starts of consecutive rows).  A matrix argument of n rows and leading
 * dimension ld must be a buffer of n*ld elements, 16-byte aligned, with ld >= n
 * and ld a multiple of 4 (FP32) or 2 (FP64).
 *
 * Errors: every call returns a status; nothing throws or aborts across the ABI.
 * Invalid arguments give HAP_E_ARG and change nothing.  A HIP failure gives
 * HAP_E_HIP with the runtime's message in hap_last_error() (per host thread);
 * after a device error the context refuses further iteration (HAP_E_STATE).
 *
 * Streams: every call is ordered on the stream given to hap_init (or to the
 * standalone call).  Calls that return a host value (iteration counts, exemplar
 * counts, net similarity, the preference) synchronise that stream.
 * One host thread at a time may use a context; separate contexts on separate
 * streams may run concurrently.
 */
#ifndef HAP_H
#define HAP_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define HAP_API __attribute__((visibility("default")))
#else
#define HAP_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hap_status;
enum {
    HAP_OK = 0,
    HAP_E_ARG = 1,          /* invalid argument; nothing was changed */
    HAP_E_DTYPE = 2,        /* unsupported data type or type combination */
    HAP_E_OOM = 3,          /* device allocation failed */
    HAP_E_HIP = 4,          /* HIP runtime error; see hap_last_error() */
    HAP_E_STATE = 5,        /* context unusable after an earlier device error */
    HAP_E_UNSUPPORTED = 6   /* size or mode not supported by the library */
};

enum { HAP_F32 = 0, HAP_F64 = 1, HAP_BF16 = 2 };

/* Similarity build modes (s_ij = -||x_i - x_j||^2, Section 2). */
enum {
    HAP_BUILD_DIRECT = 0,   /* sum of squared coordinate differences, accumulated in FP64,
                               rounded once to the output type (VALU; any d) */
    HAP_BUILD_GEMM = 1,     /* -(|x_i|^2 + |x_j|^2 - 2 x_i.x_j) with the Gram matrix on MFMA
                               in the output precision (FP32 or FP64) */
    HAP_BUILD_BF16 = 2,     /* Gram matrix on BF16 MFMA with FP32 accumulation (FP32 output) */
    HAP_BUILD_BF16X3 = 3,   /* split x = hi + lo in BF16, x.y ~ hi.hi + hi.lo + lo.hi on MFMA,
                               FP32 accumulation (FP32 output) */
    HAP_BUILD_DIRECT_L2 = 4, /* negative Euclidean distance -sqrt(sum of squared differences), the
                               similarity the paper uses for images (Section 4); FP64 sum and root,
                               rounded once (VALU; any d) */
};

/* Preference (diagonal s^l_jj) sources. */
enum {
    HAP_PREF_MEDIAN = 0,    /* median of the N(N-1) off-diagonal entries of S, every level */
    HAP_PREF_SCALAR = 1,    /* pref_scalar[l] for every point of level l */
    HAP_PREF_VECTOR = 2     /* pref_vec[l*n + j], device, in the working type */
};

/* Iteration schedules. */
enum {
    HAP_SCHEDULE_SEQUENTIAL = 0, /* Algorithm 1: the levels one after another inside an iteration */
    HAP_SCHEDULE_MRHAP = 1       /* Section 3 (MapReduce): every level from the previous iteration's
                                    state; tau and c (Eq. 2.4, 2.6) are not updated in the first
                                    iteration, phi (Eq. 2.5) uses the level above's availabilities
                                    from before the iteration's availability update */
};

typedef struct {
    uint32_t struct_size;       /* sizeof(hap_params) */
    int32_t levels;             /* L >= 1 */
    double damping;             /* lambda in [0, 1) */
    int32_t pref_mode;          /* HAP_PREF_* */
    int32_t schedule;           /* HAP_SCHEDULE_* */
    const double *pref_scalar;  /* host [levels], HAP_PREF_SCALAR only */
    const void *pref_vec;       /* device [levels*n] in the working type, HAP_PREF_VECTOR only */
    double kappa;               /* Eq. 2.7 weight in [0, 1]; 0 = the update is off (see below) */
} hap_params;

/*
 * Optional level-wise similarity update (Eq. 2.7, the optional step of Algorithm 1),
 * kappa > 0, level-sequential schedule only (hap_init rejects it with HAP_SCHEDULE_MRHAP,
 * and a kappa outside [0, 1], with HAP_E_ARG).  The maximum of Eq. 2.7 runs over j != i,
 * so it gives one value per row: level l+1 uses s^{l+1}_ij = s_ij + delta^{l+1}_i off the
 * diagonal (the diagonal keeps the preference), with
 *   delta^{l+1}_i = delta^l_i + kappa * max_{j != i}(alpha^l_ij + rho^l_ij),  delta^1 = 0,
 * computed in every iteration as the last step of level l, from that iteration's alpha^l
 * and rho^l (not accumulated over iterations).  No N x N matrix is stored; each level below
 * the top adds two row-parallel passes per iteration (3 and 2 N^2 reads).  Net similarity
 * (hap_net_similarity) is still taken on S.
 */

typedef struct hap_ctx hap_ctx;

/* Library version string, e.g. "libhap 0.1.0 gfx950". */
HAP_API const char *hap_version(void);
HAP_API const char *hap_status_string(hap_status s);
/* Message of the last failing call on this host thread ("" if none). */
HAP_API const char *hap_last_error(void);

/*
 * Similarity build, Section 2: S[i*lds + j] = -||x_i - x_j||^2 for i, j < n.
 * X: device, n x d row-major with leading dimension ldx (>= d), type x_dtype
 * (HAP_F32 or HAP_F64).  S: device, n x lds, type s_dtype.  The diagonal is
 * written as 0 and columns n..lds-1 are not touched.
 * noise_rel > 0 (FP64 output only) adds the off-diagonal tie-break noise
 * s_ij += (noise_rel * |s_ij|) * u_ij, u_ij = (splitmix64(seed ^ (i*n + j)) >> 11) * 2^-53,
 * splitmix64(x) being the first output of a SplitMix64 generator started at x.
 * Stream-ordered, does not synchronise.
 */
HAP_API hap_status hap_build_similarity(const void *X, int64_t n, int64_t d, int64_t ldx, int32_t x_dtype,
                                void *S, int64_t lds, int32_t s_dtype, int32_t build_mode,
                                double noise_rel, uint64_t seed, void *stream);

/*
 * Median of the n(n-1) off-diagonal entries of S (device, n x lds, type dtype):
 * the mean of the two middle order statistics, formed in FP64 and rounded to
 * dtype, written to *out_host as a double.  Exact (radix select on the bit
 * patterns).  2 <= n <= 65536 (HAP_E_UNSUPPORTED above: the select counts keys in
 * 32 bits).  Allocates and frees an 8 KB scratch on the stream.  Synchronises the stream.
 */
HAP_API hap_status hap_median_offdiag(const void *S, int64_t n, int64_t lds, int32_t dtype,
                              double *out_host, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid allocation): hap_median_offdiag without any allocation.  The median
 * (same value, same kernels) is written to *median_dev (device double, 8-byte aligned); the
 * call only enqueues kernels on the stream and does not synchronise.  Its radix-select state
 * lives in a static device array of 8448 bytes that the library holds on every GPU it runs on
 * until the process ends (looked up with hipGetSymbolAddress on the first call on each device,
 * so make that first call outside graph capture; the device is the current one, which must be
 * the stream's).  Every call on a GPU shares that GPU's array and
 * clears it with a kernel first, so calls that overlap on one GPU (on different streams or
 * threads) race and must not be issued.  Limits: 2 <= n <= 65536 (HAP_E_UNSUPPORTED above,
 * the array's counters are 32-bit), the layout rules of the other calls (HAP_E_ARG).
 */
HAP_API hap_status hap_median_offdiag_noalloc(const void *S, int64_t n, int64_t lds, int32_t dtype,
                                              double *median_dev, void *stream);

/*
 * Bandwidth probe for the roofline: one kernel that reads `reads` arrays in[0..reads) and writes
 * `writes` arrays out[0..writes) of rows x cols FP32 elements (device, row stride ld, 16-byte
 * aligned; cols and ld multiples of 4, cols <= 8192), with the access pattern of the sweep's
 * row pass (G = ceil(rows / rows_per_block) workgroups of 512 threads, workgroup g taking rows g,
 * g + G, g + 2G, ..., 16 bytes per thread access, every access non-temporal); each output
 * element is the sum of the inputs.  An output may be one of the inputs (the same array: each
 * element is read before it is written, by the same thread), which measures an in-place update
 * such as the row pass's of rho and alpha.  flags (a bit set) vary the pattern:
 * HAP_PROBE_CACHED loads the inputs after the first with cached loads, HAP_PROBE_BLOCKS gives
 * workgroup g the contiguous rows [g rows_per_block, (g + 1) rows_per_block); other bits are
 * rejected with HAP_E_ARG.
 * (reads, writes): (0, 1) pure write (in may be NULL; every element of a row gets the row's
 * index, the pattern of the similarity build's stores of S), (1, 0) pure read (out[0] must
 * still point at one writable element, stored to only if the data hold a marker pair, so the
 * loads cannot be dropped), (1, 1) copy, (2, 2) the
 * points-mode row pass's mix (read and write rho and alpha), (3, 2) the row pass reading S.
 * Measures what such a mix reaches on the device; not part of the method.  HAP_E_ARG for other
 * mixes or bad sizes, HAP_E_UNSUPPORTED above 8192 columns.  Stream-ordered, no synchronisation.
 */
enum { HAP_PROBE_CACHED = 1, HAP_PROBE_BLOCKS = 2 };
HAP_API hap_status hap_bandwidth_probe(int32_t reads, int32_t writes, const float *const *in, float *const *out,
                                       int64_t rows, int64_t cols, int64_t ld, int64_t rows_per_block, int32_t flags,
                                       void *stream);

/* Bytes of device workspace hap_init needs for this problem. */
HAP_API hap_status hap_workspace_size(int64_t n, int32_t levels, int32_t dtype, size_t *bytes);

/*
 * Create a context for HAP on S (device, n x lds, type dtype, n >= 2).  The
 * context borrows S: it must stay valid and unmodified until hap_destroy, and
 * its diagonal is never read or written (the preferences take its place).
 * workspace: device memory of at least hap_workspace_size() bytes, owned by the
 * caller and 256-byte aligned, or NULL for the library to allocate (and free in
 * hap_destroy).  Sets the Algorithm 1 initial state alpha = rho = 0, tau = +inf,
 * phi = c = 0 and computes the preferences.  Stream-ordered.
 */
HAP_API hap_status hap_init(hap_ctx **out, const void *S, int64_t n, int64_t lds, int32_t dtype,
                    const hap_params *params, void *workspace, size_t workspace_bytes,
                    void *stream);

/*
 * Run up to max_iters more iterations of Algorithm 1 (every level, in order,
 * per iteration).  stable_iters = K > 0 stops at the end of the first iteration
 * whose labels at every level equal those of the K previous iterations;
 * K = 0 runs exactly max_iters.  The iteration count and the stable count
 * persist across calls, so a run can be continued.  iters_done (host, may be
 * NULL) receives the total iterations completed (the stop iteration after an
 * early stop); converged (host, may be NULL) is 1 when the stable count reached
 * K.  The stop is detected one iteration late, so after an early stop the labels are
 * those of the stop iteration while the messages (hap_read_messages) are those of the
 * next one; a further call continues from there.  HAP_E_OOM if the column-partial buffer
 * the row pass needs (see hap_set_launch) cannot be allocated.  Synchronises the stream.
 */
HAP_API hap_status hap_iterate(hap_ctx *ctx, int32_t max_iters, int32_t stable_iters,
                       int32_t *iters_done, int32_t *converged);

/*
 * Exemplars of level `level` (0-based, 0 = bottom) after the last completed
 * iteration, Eq. 2.8 (lowest index on ties): labels (device int32 [n], may be
 * NULL) receives e^l_i; n_exemplars (host, may be NULL) the number of distinct
 * exemplars.  Does not change the iteration state.  Synchronises if n_exemplars.
 */
HAP_API hap_status hap_exemplars(hap_ctx *ctx, int32_t level, int32_t *labels, int32_t *n_exemplars);

/*
 * Net similarity NS^l = sum_i s^l_{i, e^l_i} (s^l_ii = p^l_i), accumulated in
 * FP64 on the GPU; level = -1 gives the sum over levels.  The paper defines no
 * objective; this is the usual affinity-propagation one (the summed similarity of
 * every point to its exemplar, an exemplar's own term being its preference).  X (device, n x d,
 * leading dimension ldx, type x_dtype) may be given to recompute the
 * similarities -||x_i - x_e||^2 in FP64 instead of reading S.  Synchronises.
 */
HAP_API hap_status hap_net_similarity(hap_ctx *ctx, int32_t level, const void *X, int64_t d, int64_t ldx,
                              int32_t x_dtype, double *out);

/* Preference p^l_0 of every level (host double [levels]).  Synchronises. */
HAP_API hap_status hap_preference(hap_ctx *ctx, double *out);

/*
 * Copy the messages of level `level` after the last completed iteration t:
 * rho^{l,t} and alpha^{l,t} into device buffers (n x ld, working type; either may
 * be NULL) and the vectors c^l, phi^l, tau^l (device [n], working type; any may
 * be NULL).  Does not change the iteration state.  For inspection and tests.
 */
HAP_API hap_status hap_read_messages(hap_ctx *ctx, int32_t level, void *rho, void *alpha, int64_t ld,
                             void *c, void *phi, void *tau);

/*
 * Eq. 2.7 row offsets delta^l of level `level` after the last completed iteration: delta
 * device [n] in the working type (all 0 at level 0, and at every level when kappa = 0).
 * Synchronises the stream.
 */
HAP_API hap_status hap_similarity_offsets(hap_ctx *ctx, int32_t level, void *delta);

/*
 * Override the sweep launch shape: threads per row (64..1024, power of two),
 * 16-byte column chunks per thread (1, 2, 4 or 8; 4 needs <= 512 threads, 8 needs
 * <= 256) and rows per workgroup (>= 1; 1 sums the column partials in row
 * order).  threads * chunks * (16 / element size) must cover n.  A shape with more
 * than min(n, 2048) workgroups (for example one row per workgroup at n > 2048) makes the
 * library allocate its own column-partial buffer of (workgroups x n) words (twice that
 * under HAP_SCHEDULE_MRHAP; 268 MB for one row per workgroup at n = 8192, FP32), kept
 * until hap_destroy; HAP_E_OOM if that allocation fails (nothing changes).  0 keeps the
 * library's choice for that field.  flags (a bit set; -1 keeps the current
 * choices): HAP_LAUNCH_STREAM selects a row pass for long rows: with 1024 threads and 1
 * to 16 chunks the streaming pass (the row is read again from the caches in its second
 * phase), with 512 threads and 16 chunks (FP32 only, n <= 32768, the default for
 * 16384 < n <= 32768) the held-row pass (the row's s and rho stay in registers between
 * the phases), with 512 (or 64) threads and 32 chunks the paired pass (FP32 only,
 * threads*64 < n <= threads*128; the default for 32768 < n <= 65536 with 128 pairs): two
 * workgroups share each block of rows_per_block rows, each holding half of every row as
 * the held-row pass does, and exchange the row maxima once per row through device memory;
 * every workgroup of the launch (2 per block, rounded up to 16) must be resident on the
 * device at once, so a shape whose grid exceeds the device's capacity returns HAP_E_ARG,
 * and if another kernel holds part of the device so that a partner never arrives, the
 * waits give up after two seconds (or HAP_PAIR_WAIT_US microseconds, read from the
 * environment when the pass is first set up) and hap_iterate returns HAP_E_HIP with the
 * context failed; without the flag the register-resident row pass; HAP_LAUNCH_EAGER issues every
 * launch from the host instead of replaying captured graphs of sweep chunks (the
 * default captures each chunk of up to 16 sweeps once on a private stream and
 * replays it on the context's stream); HAP_LAUNCH_UNFUSED keeps one row-pass launch per
 * level under the MapReduce schedule (by default, FP32 problems that read S with a
 * register-resident shape of 4 chunks per thread and 2 to 4 levels run every level of a row
 * in one launch, which reads the row of S once per sweep instead of once per level, Section
 * 3; with more workgroups than the workspace's partial rows or more than two levels its
 * column partials are library-owned, allocated on first use as above); HAP_LAUNCH_BLOCKS
 * gives workgroup g the contiguous rows [g r, (g + 1) r) (r = rows_per_block) where by
 * default, with G = ceil(rows / r) workgroups (pairs, for the paired pass), it takes rows g,
 * g + G, g + 2G, ..., so that the rows being read at any moment lie next to each other in
 * memory (the rows feeding each column partial differ; with r = 1 the two are the same).
 * Returns HAP_E_ARG
 * (and changes nothing)
 * for a shape that does not fit.  For the autotuner and for comparisons.
 */
enum { HAP_LAUNCH_STREAM = 2, HAP_LAUNCH_EAGER = 4, HAP_LAUNCH_UNFUSED = 8, HAP_LAUNCH_FUSED = 16,
       HAP_LAUNCH_BLOCKS = 32 };
HAP_API hap_status hap_set_launch(hap_ctx *ctx, int32_t threads, int32_t chunks, int32_t rows_per_block,
                                  int32_t flags);
/* The current shape and flags; flags also carries HAP_LAUNCH_FUSED (reported only, ignored by
 * hap_set_launch) when the sweeps will run the fused all-level pass. */
HAP_API hap_status hap_get_launch(hap_ctx *ctx, int32_t *threads, int32_t *chunks, int32_t *rows_per_block,
                                  int32_t *flags);

/*
 * Points mode of the register-resident row pass.  The caller states that the context's S
 * was built from X (device FP32, n x d row-major, row stride ldx; n must equal the context's
 * point count) by hap_build_similarity with HAP_BUILD_DIRECT and no noise; the row pass then
 * recomputes s_ij = -||x_i - x_j||^2 (Section 2) with the build's arithmetic (FP64
 * accumulation in coordinate order, rounded once), which gives the same values as reading S
 * and saves one N^2 read per level and iteration (about a fifth of the sweep's traffic).  The
 * one-off passes (median, labels, net similarity) and the streaming row pass still read S,
 * and so does every row pass of a context with kappa > 0.  FP32 contexts, d = 2 or 3.  X must
 * stay valid while the context iterates.  X = NULL switches the mode off.
 * Checks: n different from the context's, or a type, d or ldx that does not fit, gives
 * HAP_E_ARG / HAP_E_DTYPE / HAP_E_UNSUPPORTED before anything is launched.  Otherwise 64
 * off-diagonal entries (two corners and 62 pseudo-random pairs) are recomputed from X on the
 * device and compared bit for bit with S; any difference gives HAP_E_ARG and leaves the mode
 * as it was.  Synchronises the stream.
 */
HAP_API hap_status hap_set_points(hap_ctx *ctx, const void *X, int64_t n, int64_t d, int64_t ldx, int32_t x_dtype);

/*
 * One block of a run split by rows (the per-node message updates of Section 3, with each
 * device owning a block of rows).  Subsequent hap_iterate calls update rows [0, rows)
 * only: the row passes cover those rows, and the column sums, the availability bases and
 * tau then hold that block's contribution alone, which is what one device of a row-split
 * run computes before a collective adds the other blocks' sums.  The other rows keep
 * their messages (the initial ones, in a fresh context) and add nothing to the sums; their
 * labels and messages are not meaningful while a block is set, and the stop rule and the
 * exemplar count of hap_exemplars take rows [0, rows) only.  rows = n (the default)
 * is the whole problem.  The launch shape (rows per workgroup) applies to the block; a
 * shape that does not fit is rejected (HAP_E_ARG).  Needs the sequential schedule and
 * kappa = 0 when rows < n (HAP_E_UNSUPPORTED otherwise); HAP_E_ARG unless 1 <= rows <= n.
 */
HAP_API hap_status hap_set_row_count(hap_ctx *ctx, int64_t rows);
HAP_API hap_status hap_get_row_count(hap_ctx *ctx, int64_t *rows);

/*
 * Per-launch timing of the sweep kernels with HIP events recorded on the
 * context's stream around the launches.  enable = k >= 1 starts collecting (and
 * clears the totals) for the launches of every k-th sweep (1: every launch), 0 stops.
 * hap_profile_read returns the summed elapsed time (ms) and the count of the timed
 * launches of the row pass (Eq. 2.1-2.6 fused, one launch per level and iteration)
 * and of the column-sum epilogue (Eq. 2.4).  Timed sweeps are launched one kernel at
 * a time (never from a captured graph).  For the benchmark's roofline figure.
 */
HAP_API hap_status hap_profile(hap_ctx *ctx, int32_t enable);
HAP_API hap_status hap_profile_read(hap_ctx *ctx, double *row_pass_ms, int64_t *row_pass_launches,
                                    double *colsum_ms, int64_t *colsum_launches);

HAP_API hap_status hap_destroy(hap_ctx *ctx);

/*
 * Batched form: many independent HAP problems of up to 2048 points each (FP32), run by ONE
 * persistent kernel launch (Section 2 / Algorithm 1 on every problem; the paper's task
 * parallelism over nodes and levels, Section 3, becomes parallelism over problems and row
 * blocks).  Workgroups take work items from a queue (largest problem first): a whole problem,
 * which one workgroup runs completely (the similarity build (as HAP_BUILD_DIRECT), the median
 * preference, the Algorithm 1 initial state, the sweeps, the final labels (Eq. 2.8) and the FP64
 * net similarity), or, for problems above the split size (hap_batch_set_split), one member of
 * the gang of K workgroups that share the problem: member m sweeps a block of rows, and the gang
 * meets once per level to add the members' column sums in member order.  Problem b is point
 * rows [off_b, off_b + n[b]) of the packed X (off_b = n[0] + ... + n[b-1]).
 *
 * hap_batch_create plans the batch (offsets, queue order; no split) and copies the plan into
 * the workspace (device, hap_batch_workspace_size bytes, 256-byte aligned, owned by the
 * caller; NULL = the library allocates); it synchronises the stream.  d <= 32.
 */
typedef struct hap_batch hap_batch;
HAP_API hap_status hap_batch_workspace_size(int32_t count, const int32_t *n, int64_t d, int32_t levels,
                                            size_t *bytes);
HAP_API hap_status hap_batch_create(hap_batch **out, int32_t count, const int32_t *n /* host [count] */,
                                    int64_t d, int32_t levels, void *workspace, size_t workspace_bytes,
                                    void *stream);
/*
 * Run the whole batch: X device FP32 (sum n) x d row-major; labels device int32,
 * problem b's labels at [levels * off_b, levels * (off_b + n[b])) level-major (level l,
 * point i at levels*off_b + l*n[b] + i); net_similarity device double [count][levels+1]
 * (per level, then the total); iters device int32 [count] (iterations performed, the
 * stop iteration after an early stop).  Launches two kernels and nothing else: no
 * allocation, no copy, no synchronisation, so the call can be captured in a graph.
 * A second run of the same batch starts again from the initial state.
 * A problem run by one workgroup sums its columns in row order, so its trajectory is the
 * single-problem path's with one row per workgroup (hap_set_launch rows_per_block = 1); a
 * problem shared by a gang adds the members' row-ordered partials in member order, which is
 * the single-problem path's with rows_per_block = the gang's rows per member.  The members of a
 * gang wait for each other with a bounded wait (60 s per meeting, scaled up for runs of more
 * than 200 iterations); a gang that does not meet gives up and reports iters[b] = -1 (its labels
 * and net similarity are then not valid), and so do the gangs still running.
 */
HAP_API hap_status hap_batch_run(hap_batch *batch, const void *X, double damping, int32_t max_iters,
                                 int32_t stable_iters, int32_t *labels, double *net_similarity, int32_t *iters,
                                 void *stream);
/* Launch shape of the persistent kernel: threads per workgroup, the number of workgroups
 * (>= 1) and the row groups per workgroup.  With G row groups a workgroup sweeps G rows of
 * its problem at once (each group owning NT/G threads); the rows' column-sum contributions
 * are still added in row order, so every shape computes the same values bit for bit.
 * (threads, row_groups) is one of (256, 1), (512, 1), (512, 2), (512, 4), (1024, 4); any
 * other pair is rejected with HAP_E_ARG and changes nothing.  0 keeps the current value.
 * While some problem is split, the launch uses at most as many workgroups as fit the device
 * at once.  For the autotuner. */
HAP_API hap_status hap_batch_set_launch(hap_batch *batch, int32_t threads, int32_t workgroups, int32_t row_groups);
HAP_API hap_status hap_batch_get_launch(hap_batch *batch, int32_t *threads, int32_t *workgroups,
                                        int32_t *row_groups);
/*
 * Split large problems over gangs of workgroups: a problem of n > max(split_n, 256) points is
 * shared by K = min(max_members, ceil(n^2 / split_n^2)) workgroups, each sweeping
 * ceil(n / K) consecutive rows (K then recounted so that no member is empty).  split_n = 0
 * switches splitting off (the default); otherwise split_n >= 256; 1 <= max_members <= 16.
 * Re-plans the queue and copies it to the workspace; synchronises the stream.  Splitting
 * shortens the batch's longest item (one workgroup running the largest problem) at the cost of
 * one gang barrier per level and iteration.
 */
HAP_API hap_status hap_batch_set_split(hap_batch *batch, int32_t split_n, int32_t max_members, void *stream);
HAP_API hap_status hap_batch_get_split(hap_batch *batch, int32_t *split_n, int32_t *max_members);
/* The plan of every problem under the current split: members (host int32 [count], 1 = one
 * workgroup) and rows per member (host int32 [count]; n for a problem that is not split).
 * Either may be NULL. */
HAP_API hap_status hap_batch_get_members(hap_batch *batch, int32_t *members, int32_t *rows_per_member);
HAP_API hap_status hap_batch_destroy(hap_batch *batch);

/*
 * Learned warm start.  The paper starts every run from alpha = rho = 0 (Algorithm 1); the
 * warm start replaces only the initial availabilities.  A network predicts, per point and
 * level, y = g(v) with v = (alpha^l_jj + rho^l_jj) / |p_j| of a finished run and
 * g(v) = sign(v) (sqrt(1 + |v|) - 1).  With rho = 0, Eq. 2.2-2.3 turn a column base
 * B_j = g^-1(y) |p_j| (g^-1(y) = sign(y) |y| (|y| + 2), p the level's preference) into
 * alpha_jj = B_j and alpha_ij = min(0, B_j); every other initial value stays as in
 * Algorithm 1.
 */
#define HAP_WARM_FEATURES 32
/*
 * Per-point features of the context's S and level-1 preferences p (a = |p_i|), into F
 * (device FP32, n rows of HAP_WARM_FEATURES, row stride ldf >= HAP_WARM_FEATURES):
 *   [0,16)  the 16 largest off-diagonal s_ij of row i, descending (ties: lower j first), / a;
 *           a row with fewer than 16 off-diagonal entries repeats its smallest one
 *   16      p_i / a
 *   17      #{j != i : s_ij > p_i} / (n - 1)
 *   18      mean of the off-diagonal s_ij, / a
 *   19      log(1 + #{j != i : s_ij > p_i}) / 10
 *   20+m    log(1 + D_m) / 10, D_m = sum_{j != i} max(0, s_ij - 2^-m p_i) / a, m = 0..5
 *   26+m    (D_m(i) - M_m(i)) / max(D_m(i), M_m(i)) (0 when both are 0), M_m(i) the largest
 *           D_m(j) over the j of entries [0,16) (all j != i when n - 1 < 16)
 * Needs n >= 2 and p_i != 0.  Uses the context's column-partial buffer as scratch (no
 * iteration state is touched).  Synchronises the stream.
 */
HAP_API hap_status hap_warm_features(hap_ctx *ctx, float *F, int64_t ldf);
/*
 * Training targets of the current state: T[j*ldt + l] = g((alpha^l_jj + rho^l_jj) / |p^l_j|)
 * with alpha^l the availabilities of the last completed iteration (device FP32, n rows,
 * ldt >= levels).  Synchronises the stream.
 */
HAP_API hap_status hap_warm_targets(hap_ctx *ctx, float *T, int64_t ldt);
/*
 * Restart the context from the Algorithm 1 initial state (the preferences stay), with the
 * warm initial availabilities of the network outputs Y (device FP32, n rows, Y[j*ldy + l]
 * for level l, ldy >= levels), or the cold start when Y is NULL.  Synchronises the stream.
 */
HAP_API hap_status hap_set_warm_start(hap_ctx *ctx, const float *Y, int64_t ldy);
/*
 * Restart the context from the Algorithm 1 initial state (the preferences stay) with given
 * initial availabilities instead of alpha = 0: alpha^l_jj = alpha_diag0[j*ld + l] (device, the
 * working type, n rows, ld >= levels) and alpha^l_ij = min(0, alpha_diag0[j*ld + l]) for
 * i != j, the values Eq. 2.2-2.3 give at rho = 0 from an availability base per column (what
 * hap_set_warm_start forms from the network outputs; this call takes the values themselves,
 * for a start computed elsewhere).  HAP_E_ARG for a null pointer or ld < levels.
 * Synchronises the stream.
 */
HAP_API hap_status hap_set_warm_alpha(hap_ctx *ctx, const void *alpha_diag0, int64_t ld);
/*
 * Warm run with the cold start as fallback: hap_set_warm_start(Y), hap_iterate(max_iters,
 * stable_iters); if that run does not converge (and Y is not NULL), restart cold and iterate
 * again.  *fell_back (host, may be NULL) is 1 when the cold run's result is the one
 * returned.  stable_iters >= 1.
 */
HAP_API hap_status hap_iterate_warm(hap_ctx *ctx, const float *Y, int64_t ldy, int32_t max_iters,
                                    int32_t stable_iters, int32_t *iters_done, int32_t *converged,
                                    int32_t *fell_back);
/*
 * Warm run judged by the cold start (opt-in: it always pays for a cold run as well).  The
 * warm run from Y (hap_set_warm_start(Y), hap_iterate(max_iters, stable_iters)), then the
 * cold run (Algorithm 1's alpha = 0) on the same context; each is scored by its net
 * similarity summed over the levels (hap_net_similarity(level -1) with the X, d, ldx, x_dtype
 * given here: recomputed from X in FP64 when X is not NULL, else read from S).  The run kept
 * is the one with the larger score (the warm run on a tie), whether or not it converged: a
 * converged run can score far worse (a start from which every point stays its own exemplar
 * converges at once).  When the warm run is kept it is run again, so that the context's state and
 * labels are the kept run's (every pass is deterministic, so the rerun repeats it bit for
 * bit; HAP_E_STATE if the rerun's stop iteration differs).  Outputs (host, each may be
 * NULL): iters_done and converged of the kept run,
 * fell_back = 1 when the cold run is kept, ns_warm and ns_cold the two scores.  Y must not be
 * NULL; stable_iters >= 1.  Synchronises the stream.
 */
HAP_API hap_status hap_iterate_warm_judged(hap_ctx *ctx, const float *Y, int64_t ldy, int32_t max_iters,
                                           int32_t stable_iters, const void *X, int64_t d, int64_t ldx,
                                           int32_t x_dtype, int32_t *iters_done, int32_t *converged,
                                           int32_t *fell_back, double *ns_warm, double *ns_cold);

/*
 * The warm start's perceptron: n_in -> hidden -> hidden -> n_out, ReLU after both hidden
 * layers: h1 = relu(X W1 + b1), h2 = relu(h1 W2 + b2), y = h2 W3 + b3.  Parameters are one
 * flat FP32 device vector of hap_mlp_param_count floats: W1 (n_in x hidden, row-major), b1,
 * W2 (hidden x hidden), b2, W3 (hidden x n_out), b3.  precision HAP_F32 multiplies FP32
 * operands, HAP_BF16 rounds both operands of every product to BF16 (nearest even); both
 * accumulate in FP32 on the matrix cores.  X, Y, T are device FP32 row-major with the given
 * row strides.  The workspace (device, 256-byte aligned, caller-owned) holds the activations
 * of `rows` rows: hap_mlp_workspace_size bytes.  Nothing synchronises the stream.
 */
HAP_API int64_t hap_mlp_param_count(int32_t n_in, int32_t hidden, int32_t n_out); /* -1 for bad sizes */
HAP_API hap_status hap_mlp_workspace_size(int32_t n_in, int32_t hidden, int32_t n_out, int64_t rows, size_t *bytes);
HAP_API hap_status hap_mlp_forward(const float *params, int32_t n_in, int32_t hidden, int32_t n_out,
                                   int32_t precision, const float *X, int64_t ldx, int64_t rows, float *Y,
                                   int64_t ldy, void *workspace, size_t workspace_bytes, void *stream);
/*
 * Loss = mean over rows and outputs of (y - t)^2 (written to *loss, device double) and its
 * gradient with respect to every parameter (grad: device FP32, same layout as params).
 */
HAP_API hap_status hap_mlp_loss_grad(const float *params, int32_t n_in, int32_t hidden, int32_t n_out,
                                     int32_t precision, const float *X, int64_t ldx, const float *T, int64_t ldt,
                                     int64_t rows, float *grad, double *loss, void *workspace,
                                     size_t workspace_bytes, void *stream);
/*
 * One Adam step (Kingma and Ba, 2015) on count parameters: opt_state (device FP32, 2*count:
 * first moments, then second moments; zero before step 1), step >= 1 (bias corrections
 * 1 - beta^step).
 */
HAP_API hap_status hap_mlp_adam(float *params, const float *grad, float *opt_state, int64_t count, int64_t step,
                                double lr, double beta1, double beta2, double eps, void *stream);
/*
 * Minibatch training: step s = 0..steps-1 gathers the rows idx[s*batch .. (s+1)*batch) of
 * X and T (device int32; an index outside [0, rows) reads as NaN), computes loss and
 * gradient (loss_hist[s], device double, may be NULL) and takes Adam step step0 + s + 1
 * (beta1 0.9, beta2 0.999, eps 1e-8).  Workspace for `batch` rows.
 */
HAP_API hap_status hap_mlp_train(float *params, float *opt_state, int32_t n_in, int32_t hidden, int32_t n_out,
                                 int32_t precision, int64_t step0, const float *X, int64_t ldx, const float *T,
                                 int64_t ldt, int64_t rows, const int32_t *idx, int64_t batch, int64_t steps,
                                 double lr, double *loss_hist, void *workspace, size_t workspace_bytes,
                                 void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HAP_H */
