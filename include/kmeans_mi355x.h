/*
 * kmeans_mi355x.h -- C ABI of the MI355X (gfx950) k-means Lloyd library.
 *
 * The operation is one Lloyd iteration (S. P. Lloyd, "Least squares
 * quantization in PCM", IEEE Trans. Inf. Theory 28(2), 1982) expressed as the
 * paper's fused data-parallel loop (section 2.3: a parallel loop over the
 * sample range whose body runs once per index in no fixed order, with a
 * collect body and predicated reduce bodies; section 3.5: loops over the same
 * range fused into one pass, side-by-side reductions sharing one traversal):
 *
 *   map     for every sample i: d_ij = sum_f (x_if - c_jf)^2 for all j,
 *           L(i) = the smallest j attaining min_j d_ij            (collect)
 *   reduce  S_j = sum_{i: L(i)=j} x_i (FP64), cnt_j = |{i: L(i)=j}|,
 *           J = sum_i d_{i,L(i)} (FP64)                           (reduce)
 *   update  c_j = S_j / cnt_j rounded once to FP32 (the vector mean as sum
 *           divided by length, section 2.1); an empty cluster keeps c_j.
 *
 * Conventions for every call:
 *   - X is n x d, C is k x d, both FP32, row-major with row stride d, and
 *     16-byte aligned.  Labels are int32, counts int64, objectives FP64.
 *   - Every array argument is a DEVICE pointer owned by the caller, borrowed
 *     until the work enqueued on `stream` completes, unless marked host.
 *   - Calls are asynchronous on `stream` (NULL = the null stream): KM_OK means
 *     "enqueued".  Only kmeans_lloyd with tol >= 0 synchronises `stream`
 *     (to return iters_done).
 *   - The library never allocates device memory.  Scratch comes from a
 *     caller-provided workspace of km_plan_workspace_bytes() bytes bound with
 *     km_plan_set_workspace(), or, for kmeans_lloyd_static, from one static
 *     device array per GPU that the library's code object holds.
 *   - On any error nothing is enqueued, outputs are untouched, the status is
 *     returned and km_last_error() describes it.  No exception crosses the ABI.
 *   - Shape limits: 1 <= k <= n < 2^31, 1 <= d <= 1024.  Rows of more than
 *     128 features are assigned by a streaming pass (same distance, operation
 *     for operation) and reduced in 128-feature slices; a per-label record
 *     k * min(d, 128) * 8 bytes above 80 KiB is reduced over label chunks of
 *     44 KiB, at most 16384 of them (KM_ENOTSUP beyond).
 *   - Inputs must be finite; NaN/Inf are not checked on the hot path.
 *   - A plan is not thread-safe; distinct plans are independent.  Calls that
 *     share one plan (one workspace) must be ordered on one stream.
 *
 * Distances: the FP32 path evaluates every d_ij in direct form, features in
 * chunks of 8 accumulated by fused multiply-add, chunk partials summed by a
 * fixed pairwise tree.  Its error is at most (2 + 8 + ceil(log2(ceil(d/8))))
 * units of 2^-24 relative to d_ij, so a label can differ from the exact
 * argmin only where the top-2 distances are within that relative margin.
 * Ties go to the lowest centroid index.  Results are deterministic: the same
 * inputs on the same plan give bit-identical outputs.
 *
 * Mixed precision (KM_BF16, KM_FP8_E4M3): the matrix cores form the dense
 * -2 x.c term in the narrow format with FP32 accumulation; a per-sample error
 * band, proven from the format's unit roundoff and the norms of x and c,
 * selects the candidates that could be the FP32 path's choice, and samples
 * with more than one candidate are re-checked with the FP32 path's distance.
 * The labels therefore equal the FP32 path's bit for bit, and so do the
 * centroids; the objective comes from the FP64 per-label sums through
 * J = sum_i |x_i|^2 + sum_j (cnt_j |c_j|^2 - 2 c_j . S_j).  FP8 scales each
 * feature by a power of two s_f >= max_i |x_if| / 448 (exact) and keeps an
 * e4m3 copy of X in the workspace, made once per call; both keep a BF16 copy
 * of X (n x 16 ceil(d/16) x 2 bytes) made once per call; k <= 16384 for both
 * (KM_ENOTSUP otherwise).  Above 128 features the matrix-core operands are
 * streamed from memory through the contraction instead of being held in
 * registers and LDS.
 */
#ifndef KMEANS_MI355X_H
#define KMEANS_MI355X_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KM_OK = 0,
    KM_EINVAL = -1,      /* bad shape, null or misaligned pointer, bad value */
    KM_ENOTSUP = -2,     /* valid request the library does not implement     */
    KM_EHIP = -3,        /* a HIP runtime call failed (message has the text) */
    KM_EWORKSPACE = -4   /* no workspace bound, or it is too small           */
} km_status;

typedef enum {
    KM_FP32 = 0,         /* direct-form FP32 distances (the plain path)      */
    KM_BF16 = 1,         /* BF16 MFMA distances + proven-band FP32 recheck    */
    KM_FP8_E4M3 = 2      /* FP8 e4m3 (OCP) MFMA distances, per-feature power-
                            of-two scales + proven-band FP32 recheck          */
} km_precision;

typedef struct km_plan km_plan;

/*
 * Create a plan for n samples of dimension d and k centroids on the current
 * HIP device.  Validates the shape (KM_EINVAL) and precision (KM_ENOTSUP),
 * then queries the device (KM_EHIP without one).  *out receives the plan
 * (host memory owned by the library; free it with km_plan_destroy).
 */
km_status km_plan_create(int64_t n, int32_t d, int32_t k, km_precision prec,
                         km_plan **out);

/* Bytes of device workspace the plan needs (0 for a NULL plan). */
size_t km_plan_workspace_bytes(const km_plan *plan);

/*
 * Bind caller-owned device memory as the plan's workspace.  `ws` must be
 * 256-byte aligned and at least km_plan_workspace_bytes() long
 * (KM_EWORKSPACE otherwise).  The workspace is borrowed until the plan is
 * destroyed or another workspace is bound.  Binding a different workspace
 * drops a graph captured by km_plan_use_graphs (its kernels hold the old
 * addresses); the next kmeans_lloyd captures afresh.
 */
km_status km_plan_set_workspace(km_plan *plan, void *ws, size_t bytes);

/* Release a plan (host memory and any captured graph).  NULL is ignored. */
void km_plan_destroy(km_plan *plan);

/* Text of the last error on the calling thread ("" if none).  Valid until the
 * next library call on that thread. */
const char *km_last_error(void);

/*
 * Assign step (the map of section 2.3): for every sample, the nearest
 * centroid under squared Euclidean distance, lowest index on ties.
 *   X        [n x d] FP32 samples
 *   C        [k x d] FP32 centroids
 *   labels   [n] int32 output, L(i) in [0, k)
 *   mindist  [n] FP32 output d_{i,L(i)} as computed, or NULL
 *   objective [1] FP64 output J = sum_i d_{i,L(i)} (FP64 sum), or NULL
 * Mixed-precision plans compute labels only: mindist and objective must be
 * NULL (KM_ENOTSUP otherwise; kmeans_lloyd reports their objective).
 */
km_status kmeans_assign(km_plan *plan, const float *X, const float *C,
                        int32_t *labels, float *mindist, double *objective,
                        hipStream_t stream);

/*
 * Update step (the predicated per-label reduce of section 2.3 and the mean of
 * section 2.1) from given labels.
 *   X       [n x d] FP32 samples
 *   labels  [n] int32 labels; entries outside [0, k) are ignored, or, in the
 *           debug-validate mode of km_plan_set_validate, rejected
 *   C_old   [k x d] FP32 centroids kept for empty clusters
 *   C_new   [k x d] FP32 output: fl32(S_j / cnt_j) or C_old[j] if cnt_j = 0
 *           (may alias C_old)
 *   counts  [k] int64 output cnt_j, or NULL
 */
km_status kmeans_update(km_plan *plan, const float *X, const int32_t *labels,
                        const float *C_old, float *C_new, int64_t *counts,
                        hipStream_t stream);

/*
 * Debug-validate mode of kmeans_update (off by default).  With enable != 0,
 * kmeans_update first counts the labels outside [0, k) on the device, waits
 * on its stream for the count, and returns KM_EINVAL (nothing more enqueued,
 * outputs untouched, the count in km_last_error()) when there is any.  Off,
 * such labels are skipped without a check and the call stays asynchronous.
 */
km_status km_plan_set_validate(km_plan *plan, int32_t enable);

/*
 * Lloyd iterations, each one assign (with C_t) fused with the reduce and
 * followed by the update to C_{t+1}, all on the device.
 *   X          [n x d] FP32 samples
 *   C          [k x d] FP32 in: C_0, out: C_T
 *   labels     [n] int32 out: L_{T-1} (the labels C_T is the mean of)
 *   counts     [k] int64 out: member counts of L_{T-1}, or NULL
 *   obj_hist   [max_iter] FP64 out: J_t for t < T, or NULL
 *   max_iter   >= 1
 *   tol        < 0: run exactly max_iter iterations.
 *              >= 0: stop after iteration t >= 1 once
 *              J_{t-1} - J_t <= tol * J_{t-1} or no label changed.
 *   iters_done HOST int32 out: T, or NULL.  With tol >= 0 the call waits on
 *              `stream` to read it.
 */
km_status kmeans_lloyd(km_plan *plan, const float *X, float *C, int32_t *labels,
                       int64_t *counts, double *obj_hist, int32_t max_iter,
                       double tol, int32_t *iters_done, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as kmeans_lloyd (same arguments, kernels, launch order and results,
 * always direct launches, no timing events), but with no workspace.  The
 * plan's scratch lives in one library-owned device array of
 * KM_STATIC_SCRATCH_BYTES, allocated per device when the library's code
 * object is loaded and held until the process ends; its address is looked up
 * (hipGetSymbolAddress) on the first call on each device.  No device memory
 * is allocated or freed by the call.
 *   - The plan needs no bound workspace; one that is bound is left untouched
 *     and stays valid for kmeans_lloyd.
 *   - km_plan_workspace_bytes(plan) must be at most KM_STATIC_SCRATCH_BYTES,
 *     else KM_EWORKSPACE with nothing enqueued (64 MiB covers FP32 plans up
 *     to e.g. n = 2^20, d = k = 64; mixed-precision plans keep a copy of X
 *     in their scratch and rarely fit).
 *   - Every call on one GPU shares that GPU's array, which keeps the last
 *     call's contents (nothing in it needs to start at zero): calls that
 *     overlap in time on one GPU (other streams, other threads, other plans)
 *     race and corrupt each other's results.  Order them on one stream.
 *   - With tol >= 0 and iters_done non-NULL the call waits on `stream`, as
 *     kmeans_lloyd does (not possible under graph capture: pass NULL there).
 */
#define KM_STATIC_SCRATCH_BYTES (64u << 20)
km_status kmeans_lloyd_static(km_plan *plan, const float *X, float *C, int32_t *labels,
                              int64_t *counts, double *obj_hist, int32_t max_iter,
                              double tol, int32_t *iters_done, hipStream_t stream);

/*
 * Batched Lloyd: many independent k-means problems of different n, d and k
 * advanced together, every iteration of all of them in one launch of the
 * per-sample pass per shape class plus one finalize launch (and, with graphs
 * enabled, one graph launch for the whole call).  Each instance is the same
 * computation as kmeans_lloyd with a fixed iteration count.  Instances of
 * more than 128 features run the single-instance path (a plan of their own,
 * its workspace inside the batch's) on a stream of the batch, forked from and
 * joined back to the caller's stream within the same call.
 */
typedef struct {
    const float *X;     /* [n x d] FP32 samples (device, 16-byte aligned)       */
    float *C;           /* [k x d] FP32 in: C_0, out: C_T (device, aligned)     */
    int32_t *labels;    /* [n] int32 out: L_{T-1} (device)                      */
    int64_t *counts;    /* [k] int64 out: counts of L_{T-1}, or NULL            */
    double *obj_hist;   /* [iterations] FP64 out: J_t, or NULL                  */
    int64_t n;
    int32_t d, k;
} km_instance;

typedef struct km_batch km_batch;

/*
 * Create a batch over `count` instances (host array, copied).  Validates every
 * instance like km_plan_create (KM_EINVAL, 1 <= d <= 1024); an instance of at
 * most 128 features needs a per-label record k * d * 8 bytes of at most 80 KiB
 * (KM_ENOTSUP otherwise), a wider one whatever km_plan_create accepts.  Precision
 * KM_FP32 (direct-form FP32 distances) or KM_BF16 (BF16 MFMA distances with
 * the proven-band FP32 recheck, labels equal to the FP32 batch's), or
 * KM_FP8_E4M3, where every instance runs the single-instance FP8 path (a plan
 * each, on the batch's stream, within the call; no batched FP8 kernels).
 * Queries the device.
 */
km_status km_batch_create(const km_instance *inst, int32_t count, km_precision prec,
                          km_batch **out);
size_t km_batch_workspace_bytes(const km_batch *batch);
/* Bind device workspace (256-byte aligned, at least km_batch_workspace_bytes);
 * uploads the batch's descriptor tables (synchronous). */
km_status km_batch_set_workspace(km_batch *batch, void *ws, size_t bytes);
/*
 * Schedule: each instance's tiles of 256 samples are split into blocks of
 * `tiles_per_block` tiles (1 to 2^20, else KM_EINVAL); order 0 launches blocks
 * in instance order, order 1 by decreasing work per block.  Changes the
 * workspace size (bind a workspace again afterwards).  The autotuner in the
 * Python package picks these.
 */
km_status km_batch_set_schedule(km_batch *batch, int32_t tiles_per_block, int32_t order);
/*
 * Per-class schedules.  Instances of at most 128 features in FP32 and BF16
 * batches fall into shape classes (wider instances and FP8 batches, which run
 * per-instance plans, have none): (8-feature chunks
 * of d, LDS bucket of the FP32 fused pass's per-label record), listed in
 * increasing order; the partition does not depend on the precision, so class
 * c names the same instances in an FP32 and a BF16 batch of one instance set.
 * km_batch_num_classes counts them (0 for NULL);
 * km_batch_class_info describes class `cls` (HOST outputs, each may be NULL:
 * its chunk count, LDS bucket in bytes, number of instances, and the tiles
 * per block it currently uses); km_batch_set_class_schedule gives class `cls`
 * its own tiles per block (1 to 2^20; 0: the batch-wide value of km_batch_set_schedule,
 * which keeps setting the order).  Both setters change the workspace size:
 * bind a workspace again afterwards.
 */
int32_t km_batch_num_classes(const km_batch *batch);
km_status km_batch_class_info(const km_batch *batch, int32_t cls, int32_t *d8, int32_t *lds_bytes,
                              int32_t *instances, int32_t *tiles_per_block);
km_status km_batch_set_class_schedule(km_batch *batch, int32_t cls, int32_t tiles_per_block);
/*
 * Persistent launch (FP32 batches whose instances of at most 128 features all
 * have d <= 64; KM_ENOTSUP otherwise): kmeans_lloyd_batched then runs one
 * kernel per 32 iterations.  Its resident blocks take (iteration, work row)
 * items from a device queue in iteration order and run the fused pass; the
 * block that finishes an instance's last row of an iteration finalizes that
 * instance (the same combine order as the per-class launches, so results are
 * identical at the same schedule) and publishes its next iteration, so each
 * instance advances on its own completion ticket instead of a global
 * per-iteration barrier.  Waits are bounded: a wait past its bound sets an
 * abort flag, every block exits, and km_batch_persistent_status (synchronous)
 * reports it (*aborted = 1; the results of that call are then invalid).
 * Changes the workspace size (bind a workspace again afterwards).
 */
km_status km_batch_use_persistent(km_batch *batch, int32_t enable);
km_status km_batch_persistent_status(km_batch *batch, int32_t *aborted);
/* As km_plan_use_graphs, for kmeans_lloyd_batched (graph keyed by iterations). */
km_status km_batch_use_graphs(km_batch *batch, int32_t enable);
void km_batch_destroy(km_batch *batch);
/* `iterations` >= 1 Lloyd iterations of every instance (fixed count). */
km_status kmeans_lloyd_batched(km_batch *batch, int32_t iterations, hipStream_t stream);

/*
 * Launch mode of kmeans_lloyd.  With enable != 0 the plan captures the whole
 * call (every iteration's kernels) into a HIP graph the first time it sees a
 * given (X, C, labels, counts, obj_hist, max_iter, tol), and afterwards
 * replays that graph on the call's stream while those arguments stay the same
 * (a replay reads C afresh, so it continues from the current centroids).
 * Capture runs on a stream the plan owns, so the caller's stream may be the
 * null stream.  enable = 0 returns to direct launches and drops any graph.
 */
km_status km_plan_use_graphs(km_plan *plan, int32_t enable);

/*
 * Diagnostics: per-launch duration of the kernels that compute the
 * distances (they dominate every call): on FP32 plans the per-sample pass
 * (distances, labels and, fused, the per-label partial sums), one launch per
 * iteration; on BF16 and FP8 plans each MFMA pass, in launch order: the
 * screen, for FP8 the BF16 screen of the samples it left open, then the
 * refine (one pass per iteration for BF16 plans with k <= 128, which sweep
 * once); in gda_train, the covariance contraction.  km_plan_enable_timing(plan, cap) makes the plan record a pair
 * of HIP events on the call's stream around each such launch, for up to
 * `cap` launches (cap = 0 turns timing off and releases the events; events are
 * host-side HIP objects, no device memory is allocated).  Recording restarts
 * at every enable call.  km_plan_kernel_times() waits for the recorded events
 * and writes up to `cap` durations in milliseconds into the HOST array `ms`,
 * and the number recorded into *count.
 */
km_status km_plan_enable_timing(km_plan *plan, int32_t cap);
km_status km_plan_kernel_times(km_plan *plan, float *ms, int32_t cap,
                               int32_t *count);

/*
 * Diagnostics of a BF16 or FP8 plan: number of samples the last MFMA assign queued
 * for the exact FP32 recheck (their candidate set under the proven band had
 * more than one member), and how many of those were re-checked against all k
 * centroids because their candidate list overflowed.  Waits on `stream`;
 * writes the HOST int64 *count and *full_scans (may be NULL).  KM_EINVAL for
 * an FP32 plan.
 */
km_status km_plan_recheck_count(km_plan *plan, int64_t *count,
                                int64_t *full_scans, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Applications built from the same building blocks (paper section 4).
 */

/* Distance of kmeans_assign_metric and the applications below: sum_f |a_f - b_f| (the L1 distance of
 * the section 4.1 generated code) or sum_f (a_f - b_f)^2. */
typedef enum {
    KM_METRIC_L1 = 0,
    KM_METRIC_SQEUCLIDEAN = 1
} km_metric;

/* Sample layouts of kmeans_assign_metric. */
typedef enum {
    KM_ROW_MAJOR = 0,       /* X[i * d + f] (n x d, as everywhere else)        */
    KM_FEATURE_MAJOR = 1    /* X[f * n + i] (d x n, struct of arrays)          */
} km_layout;

/*
 * Assign step under a chosen metric and sample layout (FP32 plans;
 * KM_ENOTSUP for BF16 / FP8 plans): for every sample the nearest centroid,
 * lowest index on ties.  The squared Euclidean form is the plain path's
 * canonical distance (labels and distances bit-equal to kmeans_assign's);
 * the L1 form sums |fl(x - c)| in the same chunked order, so its error is at
 * most (1 + 8 + ceil(log2 ceil(d/8))) 2^-24 of the exact L1 distance.  Both
 * layouts give bit-identical results.
 *   X         [n x d] (row-major) or [d x n] (feature-major) FP32, 16-byte
 *             aligned
 *   C         [k x d] FP32 centroids (row-major)
 *   labels    [n] int32 output
 *   mindist   [n] FP32 output distance to the chosen centroid, or NULL
 *   objective [1] FP64 output sum of those distances, or NULL
 */
km_status kmeans_assign_metric(km_plan *plan, const float *X, km_layout layout,
                               km_metric metric, const float *C, int32_t *labels,
                               float *mindist, double *objective, hipStream_t stream);

/*
 * SPADE's density step (section 4.1, "Downsampling in Bioinformatics"): the
 * rows of the all-pairs distance matrix of X are visited in increasing index
 * order; a row whose density is already set is skipped (its distances are
 * never formed); a visited row i counts the samples j with
 * dist(i, j) < apprx_width or dist(i, j) < kernel_width (i itself included)
 * and gives that count to itself and to every sample within apprx_width whose
 * density is still unset (the first visited row to reach a sample sets it;
 * later rows never overwrite it).
 *   X              [n x d] FP32 samples, row-major (device, 4-byte aligned)
 *   apprx_width, kernel_width  thresholds (strict <), compared in FP64
 *   metric         KM_METRIC_L1 or KM_METRIC_SQEUCLIDEAN
 *   densities      [n] int32 output (device)
 *   visited        [n] int8 output (device): 1 for the visited rows, or NULL
 *   visited_count  HOST int64 output: number of visited rows, or NULL
 *   ws, ws_bytes   device workspace of spade_workspace_bytes(n, d) bytes,
 *                  256-byte aligned (no state is kept between calls)
 * Distances are evaluated in FP64 with the features summed in increasing
 * order, so every threshold decision (and every density) equals that of a
 * sequential FP64 evaluation of the same definition.  The rows are processed
 * in batches whose end the host reads back: the call waits on `stream`.
 * 1 <= n < 2^31, 1 <= d <= 1024 (KM_EINVAL otherwise); NaN widths are
 * rejected.
 */
size_t spade_workspace_bytes(int64_t n, int32_t d);
km_status spade_densities(const float *X, int64_t n, int32_t d, double apprx_width,
                          double kernel_width, km_metric metric, int32_t *densities,
                          int8_t *visited, int64_t *visited_count, void *ws,
                          size_t ws_bytes, hipStream_t stream);
/* Diagnostics of the last spade_densities call on this workspace: batches run
 * and candidate rows whose distances were formed (visited rows plus rows
 * formed speculatively inside a batch and then found claimed).  HOST outputs;
 * waits on `stream`. */
km_status spade_stats(const void *ws, int64_t n, int32_t d, int64_t *batches,
                      int64_t *candidates, hipStream_t stream);

/*
 * Per-class sums of given labels: the predicated per-label reduce of section
 * 2.3 on its own (the update step without the mean), on a plan's workspace.
 *   X       [n x d] FP32 samples (16-byte aligned)
 *   labels  [n] int32 classes in [0, k) (others are skipped, or rejected in
 *           the debug-validate mode of km_plan_set_validate)
 *   S       [k x d] FP64 output: S_cf = sum of x_if over the samples of class c
 *   counts  [k] int64 output n_c, or NULL
 * The sums are taken in a fixed order (per-block sums in sample order,
 * combined block by block), so they are deterministic; sums of integer-valued
 * features below 2^53 are exact.
 */
km_status km_class_sums(km_plan *plan, const float *X, const int32_t *labels, double *S,
                        int64_t *counts, hipStream_t stream);

/*
 * Multinomial naive Bayes training (one of the section 4.2 applications),
 * with add-one smoothing, on a plan for n samples, d features, k classes:
 *   prior  [k] FP64 output: n_c / n
 *   phi    [k x d] FP64 output: (S_cf + 1) / (T_c + d), T_c = sum_f S_cf
 *          summed in increasing f (a class without samples gets 1 / d)
 * X holds per-sample feature counts (non-negative).  labels as for
 * km_class_sums (classes must lie in [0, k)).
 */
km_status nb_train(km_plan *plan, const float *X, const int32_t *labels, double *prior,
                   double *phi, hipStream_t stream);

/*
 * Gaussian discriminant analysis training with one covariance shared by the
 * classes (one of the section 4.2 applications):
 *   prior  [k] FP64 output: n_c / n
 *   mu     [k x d] FP64 output: S_c / n_c (0 for a class without samples)
 *   sigma  [d x d] FP64 output: (1/n) sum_i z_i z_i^T, z_i = x_i - mu_{y_i}
 * The sum of outer products runs on the FP64 matrix cores in 64 x 64 output
 * regions per block of samples, the block partials combined in a fixed
 * order.  ws: device workspace of gda_workspace_bytes(plan) bytes, 256-byte
 * aligned (KM_EWORKSPACE otherwise), besides the plan's own.  labels as for
 * km_class_sums (classes must lie in [0, k)).
 */
size_t gda_workspace_bytes(const km_plan *plan);
km_status gda_train(km_plan *plan, const float *X, const int32_t *labels, double *prior,
                    double *mu, double *sigma, void *ws, size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* KMEANS_MI355X_H */
