/*
 * subkm_oracle.c -- CPU oracle for subclustered k-means.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64
 * reference of the method of "A parallel sampling based clustering"
 * (arXiv 1412.1947).  It exists to check the HIP library; only the test
 * suite, the package smoke check and the benchmark's CPU-baseline leg load
 * it.  It shares no code, header, table or helper with the HIP path.
 *
 * Build with  gcc -std=c99 -O2 -ffp-contract=off  (never -ffast-math): every
 * floating-point operation below is one IEEE-754 binary64 operation with
 * round-to-nearest-even, evaluated in the order it is written.
 *
 * What the paper leaves open is fixed as follows (the "readings"):
 *  - feature scaling is min-max scaling of every attribute to [0,1]; a
 *    constant attribute maps to 0;
 *  - the similarity to the landmark is the squared Euclidean distance
 *    (metric 0, ranks like the distance) or the Manhattan distance (metric
 *    1), the two measures Sec. II names; Lloyd is k-means, Euclidean, always;
 *  - Algorithm 1 is applied repeatedly to the points left over (Sec. II
 *    describes the recursion as "redoing the process" on the remaining points)
 *    and the landmark is recomputed over the remaining points each round;
 *    the alternative reading keeps the first landmark (fixed_landmark=1);
 *  - equal keys are broken by the lower original index, and the members of a
 *    subcluster are stored in ascending original index;
 *  - the clustering inside a subcluster is Lloyd's algorithm (Sec. I) started
 *    from the subcluster's first k points; the number of local centers of a
 *    subcluster of n_r points is ceil(n_r * k_local / N) (the compression
 *    value of Sec. VI is N / k_local);
 *  - an empty cluster keeps its center; Lloyd stops after max_iter updates or
 *    when the largest center move (Euclidean) is strictly below tol;
 *  - the final run clusters the concatenated local centers, unweighted, from
 *    the strided start C[q] = local[q * floor(M / k_final)];
 *  - Algorithm 2 (Sec. III) places its m landmarks evenly on the segment from
 *    L to H, both corner points included (p_q = L + q/(m-1) (H - L)); a point
 *    joins the nearest landmark, the lower q on a tie; groups are kept in
 *    landmark order with members in ascending index, and an empty group gets
 *    no local center.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REF_OK 0
#define REF_EINVAL 1
#define REF_ENOMEM 2

/* ------------------------------------------------------------------------ */
/* O1  Min-max feature scaling (Sec. II, Algorithm 1 step 1; Sec. III,
 *     Algorithm 2 step 1).  S may alias X.  Returns REF_EINVAL on a NaN or
 *     infinite input.                                                       */
int subkm_ref_scale(const float *X, int64_t n, int32_t d, float *S,
                    float *mins, float *maxs)
{
    if (n < 1 || d < 1) return REF_EINVAL;
    for (int32_t j = 0; j < d; ++j) {
        float mn = X[j], mx = X[j];
        for (int64_t i = 0; i < n; ++i) {
            float v = X[i * d + j];
            if (!isfinite(v)) return REF_EINVAL;
            if (v < mn) mn = v;
            if (v > mx) mx = v;
        }
        mins[j] = mn;
        maxs[j] = mx;
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t j = 0; j < d; ++j) {
            double range = (double)maxs[j] - (double)mins[j];
            if (range > 0.0) {
                double num = (double)X[i * d + j] - (double)mins[j];
                S[i * d + j] = (float)(num / range);
            } else {
                S[i * d + j] = 0.0f;
            }
        }
    }
    return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* O2  Equal sized subclustering (Sec. II, Algorithm 1).                     */

typedef struct {
    double key;
    int64_t idx;
} ref_keyed;

static int cmp_keyed(const void *a, const void *b)
{
    const ref_keyed *x = (const ref_keyed *)a, *y = (const ref_keyed *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* Similarity of row i of S to the landmark L (Sec. II leaves the measure
 * open and names the Euclidean and the Manhattan distance): metric 0 is the
 * squared Euclidean distance, metric 1 the Manhattan distance; attributes
 * taken in ascending order.                                                */
static double landmark_key(const float *row, const float *L, int32_t d, int32_t metric)
{
    double acc = 0.0;
    for (int32_t j = 0; j < d; ++j) {
        double q = (double)row[j] - (double)L[j];
        acc = acc + (metric ? fabs(q) : q * q);
    }
    return acc;
}

/* Partition the n rows of S into T = ceil(n / N) subclusters.
 * Round t: the landmark L_t is the attribute-wise minimum of the remaining
 * points (Algorithm 1 step 2); the min(N, remaining) remaining points with
 * the smallest (key, index) are gathered (step 3) and removed (step 5).
 * perm[offsets[t] .. offsets[t+1]) lists subcluster t in ascending index.
 * landmarks (nullable) receives L_t, T x d.  Returns T, or -1 on error.   */
int64_t subkm_ref_subcluster(const float *S, int64_t n, int32_t d, int64_t N,
                             int32_t fixed_landmark, int32_t metric, int64_t *perm,
                             int64_t *offsets, float *landmarks)
{
    if (n < 1 || d < 1 || N < 1 || (metric != 0 && metric != 1)) return -1;
    int64_t *rem = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *nxt = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    ref_keyed *kv = (ref_keyed *)malloc((size_t)n * sizeof(ref_keyed));
    unsigned char *taken = (unsigned char *)calloc((size_t)n, 1);
    float *L = (float *)malloc((size_t)d * sizeof(float));
    if (!rem || !nxt || !kv || !taken || !L) {
        free(rem); free(nxt); free(kv); free(taken); free(L);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) rem[i] = i;
    int64_t nrem = n, t = 0, off = 0;
    while (nrem > 0) {
        /* step 2: the landmark, recomputed over the points still left */
        if (t == 0 || !fixed_landmark) {
            for (int32_t j = 0; j < d; ++j) {
                float m = S[rem[0] * d + j];
                for (int64_t r = 1; r < nrem; ++r) {
                    float v = S[rem[r] * d + j];
                    if (v < m) m = v;
                }
                L[j] = m;
            }
        }
        if (landmarks) memcpy(landmarks + t * d, L, (size_t)d * sizeof(float));
        /* step 3: the N points closest to L */
        int64_t take = nrem < N ? nrem : N;
        for (int64_t r = 0; r < nrem; ++r) {
            kv[r].key = landmark_key(S + rem[r] * d, L, d, metric);
            kv[r].idx = rem[r];
        }
        qsort(kv, (size_t)nrem, sizeof(ref_keyed), cmp_keyed);
        for (int64_t r = 0; r < take; ++r) taken[kv[r].idx] = 1;
        /* emit the subcluster in ascending index; step 5: drop it */
        offsets[t] = off;
        int64_t left = 0;
        for (int64_t r = 0; r < nrem; ++r) {
            int64_t i = rem[r];
            if (taken[i]) perm[off++] = i;
            else nxt[left++] = i;
        }
        int64_t *sw = rem; rem = nxt; nxt = sw;
        nrem = left;
        ++t;
    }
    offsets[t] = off;
    free(rem); free(nxt); free(kv); free(taken); free(L);
    return t;
}

/* ------------------------------------------------------------------------ */
/* O2b Unequal sized subclustering (Sec. III, Algorithm 2).                  */

/* Similarity of a row of S to a binary64 landmark p (metric as for
 * landmark_key), attributes taken in ascending order.                      */
static double segment_key(const float *row, const double *p, int32_t d, int32_t metric)
{
    double acc = 0.0;
    for (int32_t j = 0; j < d; ++j) {
        double q = (double)row[j] - p[j];
        acc = acc + (metric ? fabs(q) : q * q);
    }
    return acc;
}

/* Partition the n rows of S into m groups around m landmarks placed evenly
 * on the segment between the corner points L (attribute-wise minimum, step
 * 2) and H (attribute-wise maximum, step 3):
 *     p_q[j] = L[j] + (q / (m - 1)) * (H[j] - L[j]),  q = 0 .. m-1,
 * in binary64 and in that order (q / (m - 1) first, then the product, then
 * the sum); with m = 1 the one landmark is L.  Every point joins the
 * landmark at the least squared distance, the lower q on a tie (step 5).
 * Groups are emitted in landmark order, members in ascending index; a group
 * may be empty.  perm[offsets[q] .. offsets[q+1]) lists group q.
 * landmarks (nullable) receives p, m x d binary64; group (nullable) the
 * group of every point.  Returns m, or -1 on error.                        */
int64_t subkm_ref_subcluster_unequal(const float *S, int64_t n, int32_t d, int64_t m,
                                     int32_t metric, int64_t *perm, int64_t *offsets,
                                     double *landmarks, int32_t *group)
{
    if (n < 1 || d < 1 || m < 1 || m > 0x7fffffff || (metric != 0 && metric != 1)) return -1;
    float *L = (float *)malloc((size_t)d * sizeof(float));
    float *H = (float *)malloc((size_t)d * sizeof(float));
    double *p = (double *)malloc((size_t)m * d * sizeof(double));
    int32_t *g = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t *fill = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
    if (!L || !H || !p || !g || !fill) {
        free(L); free(H); free(p); free(g); free(fill);
        return -1;
    }
    /* steps 2 and 3: the corner points */
    for (int32_t j = 0; j < d; ++j) {
        float lo = S[j], hi = S[j];
        for (int64_t i = 1; i < n; ++i) {
            float v = S[i * d + j];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
        L[j] = lo;
        H[j] = hi;
    }
    /* step 4: the landmarks along the segment from L to H */
    for (int64_t q = 0; q < m; ++q) {
        double t = m == 1 ? 0.0 : (double)q / (double)(m - 1);
        for (int32_t j = 0; j < d; ++j)
            p[q * d + j] = (double)L[j] + t * ((double)H[j] - (double)L[j]);
    }
    if (landmarks) memcpy(landmarks, p, (size_t)m * d * sizeof(double));
    /* step 5: every point to its nearest landmark */
    for (int64_t i = 0; i < n; ++i) {
        double best = segment_key(S + i * d, p, d, metric);
        int32_t bq = 0;
        for (int64_t q = 1; q < m; ++q) {
            double k = segment_key(S + i * d, p + q * d, d, metric);
            if (k < best) {
                best = k;
                bq = (int32_t)q;
            }
        }
        g[i] = bq;
    }
    if (group) memcpy(group, g, (size_t)n * sizeof(int32_t));
    /* the groups in landmark order, each in ascending index */
    for (int64_t i = 0; i < n; ++i) ++fill[g[i] + 1];
    for (int64_t q = 0; q < m; ++q) fill[q + 1] += fill[q];
    for (int64_t q = 0; q <= m; ++q) offsets[q] = fill[q];
    for (int64_t i = 0; i < n; ++i) perm[fill[g[i]]++] = i;
    free(L); free(H); free(p); free(g); free(fill);
    return m;
}

/* ------------------------------------------------------------------------ */
/* O3  Lloyd's algorithm (Sec. I names it as the clustering used inside each
 *     subcluster).  Points and centers are FP64, row-major.                 */

static double sqdist(const double *x, const double *c, int32_t d)
{
    double acc = 0.0;
    for (int32_t j = 0; j < d; ++j) {
        double q = x[j] - c[j];
        acc = acc + q * q;
    }
    return acc;
}

/* Assignment step: label = argmin_c ||x - C_c||^2, the lowest c on a tie.
 * Returns the objective sum_i min_c ||x_i - C_c||^2, summed in ascending i.
 * dmin (nullable) receives the minimum distance of each point; margin
 * (nullable) receives (D2 - D1) / D2 for the two smallest distances D1 <= D2
 * (0 when D2 == 0, +inf when k == 1).                                      */
double subkm_ref_assign(const double *X, int64_t n, int32_t d, int32_t k,
                        const double *C, int32_t *labels, double *dmin,
                        double *margin)
{
    double sse = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double *x = X + i * d;
        double best = INFINITY, second = INFINITY;
        int32_t bi = 0;
        for (int32_t c = 0; c < k; ++c) {
            double v = sqdist(x, C + (int64_t)c * d, d);
            if (v < best) {
                second = best;
                best = v;
                bi = c;
            } else if (v < second) {
                second = v;
            }
        }
        labels[i] = bi;
        sse = sse + best;
        if (dmin) dmin[i] = best;
        if (margin) {
            if (k == 1) margin[i] = INFINITY;
            else if (second > 0.0) margin[i] = (second - best) / second;
            else margin[i] = 0.0;
        }
    }
    return sse;
}

/* Update step: every center moves to the mean of its points (sums in FP64,
 * ascending i); a center with no points keeps its place.  Returns the
 * largest Euclidean center move.  counts (nullable) receives cluster sizes.
 * C_out must not alias C_in.                                               */
double subkm_ref_update(const double *X, int64_t n, int32_t d, int32_t k,
                        const int32_t *labels, const double *C_in,
                        double *C_out, int64_t *counts)
{
    double *sum = (double *)calloc((size_t)k * d, sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)k, sizeof(int64_t));
    if (!sum || !cnt) {
        free(sum); free(cnt);
        return NAN;
    }
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = labels[i];
        cnt[c] += 1;
        for (int32_t j = 0; j < d; ++j)
            sum[(int64_t)c * d + j] = sum[(int64_t)c * d + j] + X[i * d + j];
    }
    double shift = 0.0;
    for (int32_t c = 0; c < k; ++c) {
        for (int32_t j = 0; j < d; ++j) {
            int64_t e = (int64_t)c * d + j;
            C_out[e] = cnt[c] > 0 ? sum[e] / (double)cnt[c] : C_in[e];
        }
        double mv = sqrt(sqdist(C_out + (int64_t)c * d, C_in + (int64_t)c * d, d));
        if (mv > shift) shift = mv;
        if (counts) counts[c] = cnt[c];
    }
    free(sum);
    free(cnt);
    return shift;
}

/* Objective of a fixed labeling against centers C (used for the trace). */
static double labeled_sse(const double *X, int64_t n, int32_t d,
                          const int32_t *labels, const double *C)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s = s + sqdist(X + i * d, C + (int64_t)labels[i] * d, d);
    return s;
}

/* One Lloyd run from the start C0: repeat { assign; update } until max_iter
 * updates are done or the largest center move is strictly below tol; then
 * one last assignment against the returned centers gives labels and the
 * objective.  trace (nullable, 2*max_iter+1 entries) receives the objective
 * after every assignment and after every update, in order; unused entries
 * are NaN.  Returns the number of updates done, or -1 on error.           */
int32_t subkm_ref_lloyd(const double *X, int64_t n, int32_t d, int32_t k,
                        const double *C0, int32_t max_iter, double tol,
                        double *C, int32_t *labels, double *sse,
                        double *trace)
{
    if (n < 1 || d < 1 || k < 1 || k > n || max_iter < 0) return -1;
    double *nxt = (double *)malloc((size_t)k * d * sizeof(double));
    if (!nxt) return -1;
    memcpy(C, C0, (size_t)k * d * sizeof(double));
    if (trace)
        for (int32_t q = 0; q < 2 * max_iter + 1; ++q) trace[q] = NAN;
    int32_t it = 0;
    int converged = 0;
    double obj;
    for (;;) {
        obj = subkm_ref_assign(X, n, d, k, C, labels, NULL, NULL);
        if (trace) trace[2 * it] = obj;
        if (it == max_iter || converged) break;
        double shift = subkm_ref_update(X, n, d, k, labels, C, nxt, NULL);
        if (trace) trace[2 * it + 1] = labeled_sse(X, n, d, labels, nxt);
        memcpy(C, nxt, (size_t)k * d * sizeof(double));
        ++it;
        converged = shift < tol;
    }
    *sse = obj;
    free(nxt);
    return it;
}

/* ------------------------------------------------------------------------ */
/* O4  The whole two-level method (Sec. II Algorithm 1 or Sec. III
 *     Algorithm 2, and Sec. V): scale, subcluster, cluster every subcluster
 *     locally, then cluster the local centers into k_final centers; finally
 *     label all n points.
 *
 * scheme 0 subclusters with Algorithm 1 into T = ceil(n/N) subclusters of N
 * points; scheme 1 with Algorithm 2 into T = m_groups groups (m_groups = 0
 * takes ceil(n/N)).  In both, a subcluster of n_r points gets
 * ceil(n_r * k_local / N) local centers, so an empty group gets none.
 * Output capacities: S n*d; perm n; offsets T+1; local_centers at most n
 * rows; local_k, local_iters, local_sse T; centers k_final*d; labels n.
 * Centers are in scaled space.                                            */
int subkm_ref_cluster(const float *X, int64_t n, int32_t d, int64_t N,
                      int32_t k_local, int32_t k_final, int32_t max_iter,
                      double tol, int32_t fixed_landmark, int32_t scheme,
                      int64_t m_groups, int32_t metric,
                      float *S, int64_t *perm, int64_t *offsets, int64_t *T_out,
                      double *local_centers, int32_t *local_k,
                      int32_t *local_iters, double *local_sse, int64_t *M_out,
                      double *centers, int32_t *labels, double *sse,
                      int32_t *final_iters)
{
    if (n < 1 || d < 1 || N < 1 || k_local < 1 || k_local > N || k_final < 1 ||
        (scheme != 0 && scheme != 1) || m_groups < 0 || (metric != 0 && metric != 1))
        return REF_EINVAL;
    float *mins = (float *)malloc((size_t)d * sizeof(float));
    float *maxs = (float *)malloc((size_t)d * sizeof(float));
    if (!mins || !maxs) { free(mins); free(maxs); return REF_ENOMEM; }
    int rc = subkm_ref_scale(X, n, d, S, mins, maxs);
    free(mins); free(maxs);
    if (rc) return rc;

    int64_t T;
    if (scheme == 0)
        T = subkm_ref_subcluster(S, n, d, N, fixed_landmark, metric, perm, offsets, NULL);
    else
        T = subkm_ref_subcluster_unequal(S, n, d, m_groups ? m_groups : (n + N - 1) / N,
                                         metric, perm, offsets, NULL, NULL);
    if (T < 0) return REF_ENOMEM;
    *T_out = T;

    double *xr = (double *)malloc((size_t)n * d * sizeof(double));
    int32_t *lab = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!xr || !lab) { free(xr); free(lab); return REF_ENOMEM; }
    int64_t M = 0;
    for (int64_t t = 0; t < T; ++t) {
        int64_t nr = offsets[t + 1] - offsets[t];
        /* local centers of this subcluster: ceil(n_r * k_local / N) */
        int32_t kr = (int32_t)((nr * (int64_t)k_local + N - 1) / N);
        if (nr == 0) {  /* an empty group of Algorithm 2 */
            local_k[t] = 0;
            local_iters[t] = 0;
            local_sse[t] = 0.0;
            continue;
        }
        for (int64_t r = 0; r < nr; ++r)
            for (int32_t j = 0; j < d; ++j)
                xr[r * d + j] = (double)S[perm[offsets[t] + r] * d + j];
        /* start from the subcluster's first kr points */
        int32_t it = subkm_ref_lloyd(xr, nr, d, kr, xr, max_iter, tol,
                                     local_centers + M * d, lab, &local_sse[t], NULL);
        if (it < 0) { free(xr); free(lab); return REF_EINVAL; }
        local_k[t] = kr;
        local_iters[t] = it;
        M += kr;
    }
    free(xr);
    free(lab);
    *M_out = M;
    if (k_final > M) return REF_EINVAL;

    /* final run on the M local centers, strided start */
    double *c0 = (double *)malloc((size_t)k_final * d * sizeof(double));
    int32_t *flab = (int32_t *)malloc((size_t)M * sizeof(int32_t));
    if (!c0 || !flab) { free(c0); free(flab); return REF_ENOMEM; }
    int64_t stride = M / k_final;
    for (int32_t q = 0; q < k_final; ++q)
        memcpy(c0 + (int64_t)q * d, local_centers + (int64_t)q * stride * d,
               (size_t)d * sizeof(double));
    double fsse;
    int32_t fit = subkm_ref_lloyd(local_centers, M, d, k_final, c0, max_iter, tol,
                                  centers, flab, &fsse, NULL);
    free(c0);
    free(flab);
    if (fit < 0) return REF_EINVAL;
    *final_iters = fit;

    /* labels of all n points against the final centers, and their objective */
    double total = 0.0;
    double *x = (double *)malloc((size_t)d * sizeof(double));
    if (!x) return REF_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t j = 0; j < d; ++j) x[j] = (double)S[i * d + j];
        double dm;
        total = total + subkm_ref_assign(x, 1, d, k_final, centers, labels + i, &dm, NULL);
    }
    free(x);
    *sse = total;
    return REF_OK;
}
