/*
 * subkm.h -- C ABI of libsubkm, subclustered k-means on AMD Instinct MI355X
 * (gfx950).
 *
 * The method is the two-level clustering of "A parallel sampling based
 * clustering" (arXiv 1412.1947):
 *   1. feature scaling of every attribute (Sec. II, Algorithm 1 step 1),
 *      here min-max scaling to [0,1];
 *   2. equal sized subclustering (Sec. II, Algorithm 1 steps 2, 3 and 5):
 *      repeatedly gather the N remaining points closest to the landmark L,
 *      the point made of the attribute-wise minima of the remaining points;
 *   3. Lloyd's k-means inside every subcluster (Algorithm 1 step 4; Sec. I
 *      names Lloyd's algorithm), giving the local centers;
 *   4. Lloyd's k-means on the local centers to obtain the required number of
 *      centers (Sec. I, Sec. V).
 *
 * Conventions shared by every call:
 *  - Points are row-major n x d float32 arrays ("row major flattening",
 *    Sec. V): the d attributes of a point are contiguous.
 *  - Every array argument is a DEVICE pointer (memory of the context's GPU,
 *    e.g. a torch CUDA tensor) unless the comment says "host".  The caller
 *    owns every input and output buffer; the library owns only its context
 *    and the scratch memory the context keeps between calls.
 *  - Calls are asynchronous on the context's stream unless stated otherwise:
 *    outputs are valid once that stream has been synchronised.  Inputs must
 *    stay valid until then.
 *  - Every call returns a status and never aborts or throws.  Arguments are
 *    validated before any device work; on an error status the outputs are
 *    unspecified and subkm_last_error() describes the problem.
 *  - One context per host thread; calls on one context must not overlap.
 */
#ifndef SUBKM_H
#define SUBKM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SUBKM_OK = 0,
    SUBKM_EINVAL = 1,      /* invalid argument (or non-finite input data)      */
    SUBKM_ENOMEM = 2,      /* device scratch memory could not be allocated     */
    SUBKM_EDEVICE = 3,     /* a HIP runtime call failed                         */
    SUBKM_EBUSY = 4,       /* serving engine full or over its memory budget    */
    SUBKM_EUNSUPPORTED = 5 /* combination of arguments not supported            */
} subkm_status;

typedef struct subkm_ctx subkm_ctx;

/* Create a context on HIP device `device`, issuing work on `stream` (a
 * hipStream_t; NULL selects the device's null stream).  *out receives the
 * context.  The stream must outlive the context or be replaced first.      */
subkm_status subkm_create(int device, void *stream, subkm_ctx **out);

/* Destroy a context and free its scratch memory (synchronises its stream). */
void subkm_destroy(subkm_ctx *ctx);

/* Text of the last error on this context ("" if none).  Valid until the
 * next call on the same context.  NULL ctx gives the last create error.     */
const char *subkm_last_error(const subkm_ctx *ctx);

/* Replace the stream of a context (hipStream_t, NULL = null stream).        */
subkm_status subkm_set_stream(subkm_ctx *ctx, void *stream);

/* Block the host until all work issued on the context's stream is done.
 * Returns SUBKM_EDEVICE when a persistent Lloyd launch issued since the
 * last such report gave up waiting at one of its barriers (a bounded spin
 * that a device running the whole cooperative grid never exhausts); the
 * results of that subkm_lloyd_batched or subkm_cluster call are invalid.  */
subkm_status subkm_synchronize(subkm_ctx *ctx);

/* ---------------------------------------------------------------------- */
/* Min-max feature scaling (Sec. II, Algorithm 1 step 1; Sec. III,
 * Algorithm 2 step 1).
 *
 * For every attribute j: mins[j] = min_i X[i][j], maxs[j] = max_i X[i][j]
 * (exact float32), and S[i][j] = (float)(((double)X[i][j] - mins[j]) /
 * ((double)maxs[j] - mins[j])) with binary64 subtraction and division,
 * rounded once to float32; an attribute with maxs[j] == mins[j] maps to 0.
 *
 * X: n x d input.  S: n x d output, may alias X.  mins, maxs: d outputs.
 * Requires n >= 1, 1 <= d.  A NaN or infinite input value gives
 * SUBKM_EINVAL; this check needs the results of the min/max pass, so the
 * call synchronises the stream once.                                      */
subkm_status subkm_scale(subkm_ctx *ctx, const float *X, int64_t n, int32_t d,
                         float *S, float *mins, float *maxs);

/* subkm_scale without any allocation, for callers that cannot allocate
 * memory: code inside HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, arithmetic, bits and errors as
 * subkm_scale; it calls no hipMalloc, hipFree or other allocating routine
 * and leaves the context's scratch untouched (subkm_device_bytes does not
 * change).  Its scratch -- the non-finite flag and the per-block min/max
 * partials -- is one static device array of 4 MiB that every GPU the
 * library runs on holds from the library's first use there until the
 * process ends; its per-device address is looked up when a context is
 * created.  The grid of the min/max pass is capped so that its partials
 * always fit (2 d floats per block), so every n and d that subkm_scale
 * accepts fits; a shape that did not would be refused with SUBKM_EINVAL.
 * The array is shared by all calls on one GPU and keeps the last call's
 * contents: calls that overlap on one GPU (two contexts or streams of the
 * same device) race and must be serialised by the caller.  Like subkm_scale
 * it synchronises the stream once (the non-finite check), so it cannot be
 * captured into a graph itself.                                          */
subkm_status subkm_scale_noalloc(subkm_ctx *ctx, const float *X, int64_t n, int32_t d,
                                 float *S, float *mins, float *maxs);

/* Min-max scaling of a column-major X (Sec. V flattens the data row by row
 * or column by column; this is the column-major input): attribute j of point
 * i at X[j * n + i].  S, mins, maxs and the arithmetic are those of
 * subkm_scale (S row-major n x d), so both layouts give the same bits.
 * S must not alias X.                                                      */
subkm_status subkm_scale_colmajor(subkm_ctx *ctx, const float *X, int64_t n, int32_t d,
                                  float *S, float *mins, float *maxs);

/* ---------------------------------------------------------------------- */
/* Similarity to a landmark (Sec. II leaves the measure open and names the
 * Euclidean and the Manhattan distance).  It only decides the subclusters;
 * the clustering inside them is k-means (squared Euclidean) either way.   */
#define SUBKM_METRIC_L2 0 /* squared Euclidean distance (ranks as Euclidean) */
#define SUBKM_METRIC_L1 1 /* Manhattan distance                            */

/* ---------------------------------------------------------------------- */
/* Equal sized subclustering (Sec. II, Algorithm 1 steps 2, 3 and 5, applied
 * round after round to the points left over).
 *
 * Round t (t = 0 .. T-1, T = ceil(n / N)):
 *   L_t[j] = min over the remaining points of S[i][j]   (landmark_mode 0),
 *            or the first landmark L_0 in every round     (landmark_mode 1);
 *   key_i  = sum_j ((double)S[i][j] - (double)L_t[j])^2     (SUBKM_METRIC_L2)
 *         or sum_j |(double)S[i][j] - (double)L_t[j]|       (SUBKM_METRIC_L1),
 *            binary64, j ascending, no fused multiply-add;
 *   G_t    = the min(N, remaining) remaining points with the smallest
 *            (key_i, i) in lexicographic order (ties to the lower index);
 *   G_t is written in ascending index to perm[t*N ..] and its rows to P.
 *
 * S: n x d input (normally the output of subkm_scale).
 * P: n x d output, P[r] = S[perm[r]] (subcluster t occupies rows
 *    offsets[t] .. offsets[t+1]-1).
 * perm: n int32 output.  offsets: T+1 int64 output; offsets[t] = t*N for
 * t < T and offsets[T] = n.  landmarks: nullable, T x d float32 output of
 * the landmarks L_t.
 * Requires 1 <= n < 2^31, 1 <= d <= 4096, N >= 1.  The selection is exact:
 * perm and P equal those of a sort by (key, index) bit for bit.          */
subkm_status subkm_subcluster(subkm_ctx *ctx, const float *S, int64_t n, int32_t d,
                              int64_t N, int32_t landmark_mode, int32_t metric, float *P,
                              int32_t *perm, int64_t *offsets, float *landmarks);

/* ---------------------------------------------------------------------- */
/* Unequal sized subclustering (Sec. III, Algorithm 2).
 *
 *   L[j] = min_i S[i][j],  H[j] = max_i S[i][j]        (steps 2 and 3);
 *   p_q[j] = (double)L[j] + (q / (double)(m - 1)) * ((double)H[j] - (double)L[j]),
 *            q = 0 .. m-1, binary64 in that order; p_0 = L when m = 1
 *            (step 4: m landmarks evenly on the segment, both ends included);
 *   group_i = argmin_q sum_j ((double)S[i][j] - p_q[j])^2   (SUBKM_METRIC_L2)
 *          or argmin_q sum_j |(double)S[i][j] - p_q[j]|     (SUBKM_METRIC_L1),
 *            binary64, j ascending, no fused multiply-add, the lower q on a
 *            tie (step 5).
 * Group q is written in ascending index to perm[offsets[q] .. offsets[q+1])
 * and its rows to the same rows of P; a group may be empty.
 *
 * S: n x d input (normally the output of subkm_scale), finite values.
 * P: n x d output, P[r] = S[perm[r]].  perm: n int32 output.  offsets: m+1
 * int64 output (offsets[0] = 0, offsets[m] = n).  landmarks: nullable,
 * m x d binary64 output of p_q.
 * Requires 1 <= n < 2^31, 1 <= d <= 4096, 1 <= m <= 8192.  The result is
 * the argmin over all m landmarks bit for bit; the search visits only the
 * few landmarks near each point's projection on the segment and proves the
 * rest farther with a rounding-error bound.                              */
subkm_status subkm_subcluster_unequal(subkm_ctx *ctx, const float *S, int64_t n, int32_t d,
                                      int64_t m, int32_t metric, float *P, int32_t *perm,
                                      int64_t *offsets, double *landmarks);

/* ---------------------------------------------------------------------- */
/* Many independent Lloyd runs in one call (Sec. II Algorithm 1 step 4 for
 * every subcluster; Sec. V runs every subcluster on its own block of
 * threads).
 *
 * Run r clusters runs[r].n points of runs[r].d attributes, stored row-major
 * at P + runs[r].x_off, into runs[r].k centers stored at C + runs[r].c_off;
 * C holds the starting centers on entry and the result on return.  Every
 * run repeats { assign every point to its nearest center (ties to the lower
 * center index); move every center to the mean of its points (a center with
 * no point stays) } until max_iter moves were made or the largest Euclidean
 * center move of the run is strictly below tol; a last assignment against
 * the returned centers gives labels[runs[r].lab_off + i] (center index
 * within the run) and sse[r] = sum_i min_c ||x_i - C_c||^2 (binary64).
 * iters[r] receives the number of moves made.
 *
 * runs: HOST array of R descriptors.  P, C, labels: device buffers holding
 * every run at the given offsets (runs must not overlap in C or labels).
 * iters (R int32) and sse (R double): device outputs.
 *
 * precision: the arithmetic of the first distance pass.
 *            SUBKM_PREC_FP32: float32 products, except in runs whose
 *            centers fit on chip with 8, 16 or 32 attributes, where each
 *            product is the sum of the four products of split bfloat16
 *            pairs (x = x_hi + x_lo, both operands), accumulated in float32
 *            on the matrix cores (relative error about 2^-16), and in runs
 *            of 32 attributes and at most 1024 centers whose centers do not
 *            fit on chip, which take the split form with three products per
 *            pair (the smallest dropped);
 *            SUBKM_PREC_BF16: additionally that three-product split form
 *            for such runs of 33 to 128 attributes.  In both,
 *            every point whose two nearest centers are closer than the
 *            error bound of the arithmetic used is re-assigned (float32,
 *            then binary64 distances), so the labels are those of exact
 *            arithmetic on the float32 inputs and both settings give the
 *            same results.  Center sums are exact (64-bit fixed point), so
 *            results do not depend on the order of the work.
 * form:      SUBKM_FORM_BATCHED runs every run together (one launch per
 *            phase for all runs); SUBKM_FORM_PLAIN runs one run at a time
 *            with one launch per phase and run (the reference form).  Both
 *            give identical results.
 * Requires R >= 1, n >= 1, 1 <= d <= 4096, 1 <= k <= n per run,
 * max_iter >= 0, tol >= 0.
 *
 * The call never synchronises the stream (with tuning on, the first call
 * of a new shape does; see below).  The run descriptors are staged through
 * a ring of pinned host buffers, so `runs` may be reused as soon as the
 * call returns; a call waits only when the copy issued from the same ring
 * slot four calls earlier has not run yet.  A persistent launch that gives
 * up at a barrier is reported by the next subkm_synchronize.              */
typedef struct {
    int64_t x_off;   /* offset of the run's first point in P, in floats      */
    int64_t n;       /* number of points                                     */
    int64_t c_off;   /* offset of the run's first center in C, in floats     */
    int64_t lab_off; /* offset of the run's first label in labels           */
    int32_t d;       /* attributes                                           */
    int32_t k;       /* centers                                              */
} subkm_run;

#define SUBKM_PREC_FP32 0
#define SUBKM_PREC_BF16 1
#define SUBKM_FORM_BATCHED 0
#define SUBKM_FORM_PLAIN 1

subkm_status subkm_lloyd_batched(subkm_ctx *ctx, const float *P, const subkm_run *runs,
                                 int32_t R, float *C, int32_t *labels, int32_t max_iter,
                                 double tol, int32_t precision, int32_t form,
                                 int32_t *iters, double *sse);

/* ---------------------------------------------------------------------- */
/* Schedule tuner of the batched form (Sec. V runs the subclusters in
 * parallel; how the runs of a call share the device is this library's
 * choice).  The schedule is the persistent kernel's grid, the largest
 * number of blocks that split one run (up to 128), the fewest 256-point
 * tiles such a block takes per move (1 or 2: more blocks per run shorten a
 * move's tiles, fewer shorten its barriers), and how such blocks combine
 * their sums every move (each publishes its part and sums a slice of all
 * parts, two barriers; or each adds its part into shared totals with
 * integer atomics, one barrier); it changes no result (sums are
 * exact integers, labels exact), only the time.  With tuning on, the first
 * batched call with moves of a new shape (number of runs, points, smallest
 * and largest d and k, precision) runs itself under each candidate schedule
 * on the caller's data, restarting from the caller's centers, keeps the
 * fastest for the shape, and returns the result of one more run with it
 * (such a tuning call synchronises the stream after every candidate).
 * Tuned schedules are used whether tuning is on or off.
 *   subkm_tune_enable: on = 1 tunes unseen shapes, 0 stops (default 0).
 *   subkm_tune_count: number of tuned shapes.
 *   subkm_tune_save / _load: the tuned schedules as a text file (load adds
 *   to the context's schedules; SUBKM_EINVAL on a malformed file; files of
 *   the earlier formats load: without the exchange field with published
 *   parts, without the tiles field also with 2 tiles).                  */
subkm_status subkm_tune_enable(subkm_ctx *ctx, int32_t on);
subkm_status subkm_tune_count(subkm_ctx *ctx, int32_t *entries);
subkm_status subkm_tune_save(subkm_ctx *ctx, const char *path);
subkm_status subkm_tune_load(subkm_ctx *ctx, const char *path);

/* ---------------------------------------------------------------------- */
/* The whole two-level method (Sec. II Algorithm 1 or Sec. III Algorithm 2,
 * and Sec. V): scale X, subcluster it (Algorithm 1: subclusters of N points;
 * Algorithm 2, opts->scheme = SUBKM_SCHEME_UNEQUAL: opts->m groups, or
 * ceil(n / N) when opts->m is 0), run Lloyd in every non-empty subcluster
 * with k_r = ceil(n_r * k_local / N) centers started from the subcluster's
 * first k_r points (the compression value of Sec. VI is N / k_local), then
 * run Lloyd on the M = sum_r k_r local centers with k_final centers started
 * from local center q * floor(M / k_final) for q = 0 .. k_final-1, and label
 * every point.
 *
 * X: n x d input (not modified), row-major, or column-major with
 * opts->layout = SUBKM_LAYOUT_COL.  centers: k_final x d output, in scaled
 * space (unscale with the mins/maxs of subkm_scale).  labels: n int32
 * output, the final center of every point in input order.  sse: 1 double
 * output, sum over all points of the squared distance to its final center,
 * in scaled space.  opts: nullable.  stats: nullable HOST output; when given
 * the call synchronises at its end, reports phase times, and reports a
 * persistent Lloyd barrier that gave up as subkm_synchronize does.
 * Host round trips: the call synchronises the stream once after the
 * min/max pass (the non-finite check of subkm_scale), once more at the end
 * when stats is given, and with Algorithm 2 once to read the group sizes;
 * it makes no other.
 * Requires k_local <= N and k_final <= M, besides the requirements of the
 * calls above.  With Algorithm 2, T = m and M depends on the group sizes:
 * M <= min(n, floor(n * k_local / N) + m) (the capacity opts->local_centers
 * needs), and k_final > M is found, and reported as SUBKM_EINVAL, only
 * after the groups are formed; the call then synchronises once to read the
 * group sizes.                                                            */
#define SUBKM_LAYOUT_ROW 0     /* X row-major, n x d (default)               */
#define SUBKM_LAYOUT_COL 1     /* X column-major: X[j * n + i]               */
#define SUBKM_SCHEME_EQUAL 0   /* Algorithm 1 (default) */
#define SUBKM_SCHEME_UNEQUAL 1 /* Algorithm 2 */

typedef struct {
    int32_t landmark_mode; /* 0: landmark recomputed each round (default)   */
    int32_t precision;     /* SUBKM_PREC_*                                   */
    int32_t form;          /* SUBKM_FORM_* of the local runs                 */
    int32_t scheme;        /* SUBKM_SCHEME_*                                 */
    /* optional device outputs of intermediates (NULL = not wanted) */
    float *S;              /* n x d scaled points                            */
    int32_t *perm;         /* n, subcluster order                            */
    float *local_centers;  /* M x d                                          */
    int32_t *local_iters;  /* T                                              */
    double *local_sse;     /* T                                              */
    int64_t m;             /* Algorithm 2: groups (0: ceil(n / N))           */
    int32_t metric;        /* SUBKM_METRIC_* of the subclustering            */
    int32_t layout;        /* SUBKM_LAYOUT_* of X                            */
} subkm_opts;

typedef struct {
    int64_t T;               /* subclusters                                   */
    int64_t M;               /* local centers                                 */
    int32_t final_iters;     /* moves of the final run                        */
    int32_t sub_selections;  /* Algorithm 1: selection passes of the
                                subclustering, T - 1 when every round selects
                                on its own, fewer when consecutive rounds
                                share a landmark and one pass selects all
                                their subclusters; 0 with Algorithm 2        */
    int64_t local_point_iters; /* sum over local runs of n_r * iters_r        */
    int64_t final_point_iters; /* M * final_iters                             */
    double us_scale;         /* phase times, microseconds (device events)     */
    double us_subcluster;
    double us_local;
    double us_final;
    double us_label;
    double us_total;
    int64_t rechecked;       /* point assignments redone in binary64 (local +
                                final + labelling passes)                     */
} subkm_stats;

subkm_status subkm_cluster(subkm_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t N,
                           int32_t k_local, int32_t k_final, int32_t max_iter, double tol,
                           const subkm_opts *opts, float *centers, int32_t *labels,
                           double *sse, subkm_stats *stats);

/* Sizes of the two-level problem with Algorithm 1: T = ceil(n / N)
 * subclusters and M = sum_r ceil(n_r * k_local / N) local centers (host
 * only, no device work).  Returns SUBKM_EINVAL on invalid sizes.          */
subkm_status subkm_cluster_sizes(int64_t n, int64_t N, int32_t k_local,
                                 int64_t *T, int64_t *M);

/* Device memory a subkm_cluster call of these sizes needs besides its
 * inputs and outputs, in bytes (host only): an upper bound of the scratch
 * the call adds to a fresh context, for either precision and form, with
 * Algorithm 1 (the scheme the serving engine runs).  Used for admission
 * control.  Returns 0 for invalid sizes.                                  */
size_t subkm_cluster_footprint(int64_t n, int32_t d, int64_t N, int32_t k_local,
                               int32_t k_final);

/* Device memory the context holds as scratch right now, in bytes (host
 * only; scratch grows to the largest call and is kept until destroy).     */
size_t subkm_device_bytes(const subkm_ctx *ctx);

/* ---------------------------------------------------------------------- */
/* Serving: an engine on one device takes whole clustering jobs (the method
 * of subkm_cluster) as they arrive, admits them in arrival order when one of
 * its `slots` is idle and the device memory the job adds keeps the engine
 * within `budget_bytes`, and runs admitted jobs concurrently on separate
 * streams; a job's points are copied in and its results copied out by the
 * engine (host buffers; pinned memory lets the copies overlap other jobs).
 * The points of a job stay resident on the device while it runs.
 *
 * subkm_engine_submit returns at once with a job id (SUBKM_ENOMEM when the
 * job could never fit the budget, SUBKM_EINVAL for invalid sizes).
 * subkm_engine_wait blocks until the job is done; subkm_engine_poll does not
 * block.  Both release the job's record once they report it done; a wait
 * whose record another thread released meanwhile returns SUBKM_EINVAL.
 * Results do not depend on which other jobs run at the same time.  destroy
 * waits for running jobs, cancels the waiting ones (status SUBKM_EBUSY),
 * wakes every thread blocked in subkm_engine_wait and returns only after
 * they have left it.  The engine itself is thread safe.                  */
typedef struct subkm_engine subkm_engine;

typedef struct {
    const float *X;    /* HOST n x d input, row-major, valid until the job ends */
    int64_t n;
    int64_t N;         /* subcluster size                                    */
    int32_t d;
    int32_t k_local;
    int32_t k_final;
    int32_t max_iter;
    double tol;
    int32_t precision; /* SUBKM_PREC_*                                       */
    int32_t reserved;
    float *centers;    /* HOST output, k_final x d (scaled space)            */
    int32_t *labels;   /* HOST output, n; may be NULL                        */
} subkm_job;

typedef struct {
    int32_t status;       /* subkm_status of the job                         */
    int32_t slot;         /* slot that ran it                                */
    double sse;           /* objective over all points (scaled space)        */
    double t_submit;      /* seconds on the engine's clock                   */
    double t_admit;
    double t_start;
    double t_done;        /* results are in the host buffers                 */
    size_t footprint;     /* device bytes the job needs on an empty slot     */
    size_t device_bytes;  /* device bytes the engine held when it finished   */
    size_t slot_bytes_admitted; /* the slot's device bytes allowed for the job */
    size_t slot_bytes_after;    /* the slot's device bytes after the job       */
    char message[128];    /* error text when status != SUBKM_OK              */
} subkm_job_result;

subkm_status subkm_engine_create(int device, size_t budget_bytes, int32_t slots,
                                 subkm_engine **out);
void subkm_engine_destroy(subkm_engine *e);
const char *subkm_engine_last_error(const subkm_engine *e);
size_t subkm_job_footprint(const subkm_job *job);
subkm_status subkm_engine_submit(subkm_engine *e, const subkm_job *job, int64_t *id);
subkm_status subkm_engine_poll(subkm_engine *e, int64_t id, int32_t *done, subkm_job_result *res);
subkm_status subkm_engine_wait(subkm_engine *e, int64_t id, subkm_job_result *res);
subkm_status subkm_engine_stats(subkm_engine *e, int32_t *queued, int32_t *running,
                                size_t *device_bytes);

/* ---------------------------------------------------------------------- */
/* Per-launch kernel timing (diagnostics; not part of the method).
 * When enabled, the library records a pair of HIP events on the context's
 * stream around every launch of each kernel class below and accumulates
 * the elapsed device time.  Enabling (or disabling) resets the counters.
 * subkm_profile_query synchronises the stream and returns the number of
 * launches and their total milliseconds for one class.
 * Classes: 0 assign, 1 update, 2 keys, 3 cand, 4 scatter, 5 scale,
 * 6 lloyd_fused, 7 subcluster (see subkm_profile_name).  The subclustering
 * rounds run as one replayed HIP graph, timed as a whole under class 7;
 * classes 2-4 then stay empty.                                            */
subkm_status subkm_profile_enable(subkm_ctx *ctx, int32_t on);
subkm_status subkm_profile_query(subkm_ctx *ctx, int32_t cls, int64_t *launches, double *ms);
const char *subkm_profile_name(int32_t cls);

#ifdef __cplusplus
}
#endif

#endif /* SUBKM_H */
