// Device-side types and helpers shared by the Lloyd kernels (lloyd.hip: runs
// whose centers fit on chip; lloyd_wide.hip: runs whose centers stream from
// memory).  Not part of the C ABI.
#pragma once

#include "internal.h"

#pragma clang fp contract(off)

namespace subkm_lloyd {

constexpr int kAT = 256;  // threads per block = points per assignment tile
constexpr int kWalkD = 128;            // widest points of the balanced update walk
constexpr int kWalkW = 256;            // positions per wavefront in the walk
constexpr int kWalkB = 4 * kWalkW;     // positions per walk item (block), 64-lane groups
constexpr int kWalkCenters = 256;      // centers per update item of a walked run

// Fewest lanes that hold one point in the walk: the next power of two >= d,
// at most 64 (wider points take two attributes per lane).  A wavefront holds
// DevRun::wpp points side by side (at most 64 / walk_lanes(d)), each group of
// 64 / wpp lanes walking its own window of kWalkW positions, so a walk item
// spans kWalkB * wpp positions.
__host__ __device__ inline int walk_lanes(int d) {
    int g = 1;
    while (g < d && g < 64) g <<= 1;
    return g;
}

enum : int32_t { PH_ITER = 0, PH_FINAL = 1, PH_DONE = 2 };

// One Lloyd run as the kernels see it (offsets in elements).
struct DevRun {
    int64_t x_off, n, c_off, lab_off;
    int32_t d, k;
    int32_t item0, nitems;    // assignment items (tiles of kAT points) of the run
    int32_t uitem0, nuitems;  // update items (chunks of centers)
    int32_t kcu;              // centers per update item
    int32_t fused;            // k*d fits the on-chip sums (one-block update)
    int64_t sum_off;          // on-chip path: the run's int64 sums (k*d) + counts (k)
    int64_t part_off;         // batched on-chip form: the run's exchange slots
    int32_t G;                // batched on-chip form: blocks of the run
    int32_t mf;               // assignment on matrix cores
    int64_t box_off;          // the run's attribute minima and maxima (ordered bits)
    int64_t cnt_off;          // wide path: counts | starts | cursors (3 k int32)
    int64_t frag_off;         // split-bfloat16 path: center fragments (uint4 units)
    int64_t cn_off;           // split-bfloat16 path: squared norms of the centers
    int32_t split;            // assignment with split-bfloat16 products
    int32_t orig;             // index of the run in the caller's array
    int32_t xatom;            // batched on-chip form: partial sums added into shared totals
    int32_t wpp;              // wide path, d <= kWalkD: points per wavefront in the update walk
    int32_t pad;
};

struct RunState {
    int32_t phase;
    int32_t iters;
    uint32_t ucount;
    uint32_t arrive;
    unsigned long long shift_bits;
    unsigned long long rechecks;
    uint32_t absmax_bits;
    uint32_t pad;
    unsigned long long rc2_bits;  // split path: max_c ||c - m||^2 (binary64 bits)
};

struct Item {
    int32_t run;
    int32_t first;  // first point (assignment) or first center (update)
    int32_t slice;
    int32_t pad;
};

struct Task {
    int32_t run;
    int32_t g;  // part g of the run's G blocks
};

// The value of lane l ^ 16 (lane_xor16) or l ^ 32 (lane_xor32) of the
// wavefront, from the gfx950 row swaps: permlane16_swap(x, x) returns
// (rows 0, 0, 2, 2) and (rows 1, 1, 3, 3) of x, permlane32_swap(x, x) the
// lower and the upper half twice; each lane takes the copy of its partner.
// No LDS round trip, unlike a general shuffle.  Every lane must be active.
__device__ __forceinline__ uint32_t lane_xor16(uint32_t x) {
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return ((threadIdx.x >> 4) & 1u) ? r[0] : r[1];
}
__device__ __forceinline__ uint32_t lane_xor32(uint32_t x) {
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return ((threadIdx.x >> 5) & 1u) ? r[0] : r[1];
}
__device__ __forceinline__ float lane_xor16(float x) { return __uint_as_float(lane_xor16(__float_as_uint(x))); }
__device__ __forceinline__ float lane_xor32(float x) { return __uint_as_float(lane_xor32(__float_as_uint(x))); }
__device__ __forceinline__ int32_t lane_xor16(int32_t x) { return (int32_t)lane_xor16((uint32_t)x); }
__device__ __forceinline__ int32_t lane_xor32(int32_t x) { return (int32_t)lane_xor32((uint32_t)x); }

// Exact binary64 distance of a float32 point to a float32 center, attributes
// left to right, separate multiply and add: the arithmetic of the objective.
__device__ __forceinline__ double dist64(const float *x, const float *c, int d) {
    double acc = 0.0;
    for (int j = 0; j < d; ++j) {
        double q = (double)x[j] - (double)c[j];
        acc = acc + q * q;
    }
    return acc;
}

// Binary64 argmin over all k centers of one point, by one wavefront: lanes
// take centers lane, lane+64, ...; ties go to the lowest index.
__device__ __forceinline__ int32_t wave_argmin64(const float *x, const float *C, int d, int k) {
    const int lane = threadIdx.x & 63;
    double best = INFINITY;
    int32_t bi = 0x7fffffff;
    for (int c = lane; c < k; c += 64) {
        double v = dist64(x, C + (int64_t)c * d, d);
        if (v < best) {
            best = v;
            bi = c;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        double ob = __shfl_xor(best, o, 64);
        int32_t oi = __shfl_xor(bi, o, 64);
        if (ob < best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
        }
    }
    return bi;
}

// Label bits of a run with k centers (ballot rounds of wave_count_add).
__device__ __forceinline__ int label_bits(int k) { return k > 1 ? 32 - __clz(k - 1) : 0; }

// counter[l] += 1 for every active lane with label l, with one atomic per
// distinct label of the wavefront: lanes with equal labels are matched by
// ballots over the nbits label bits, and the lowest lane of each group adds
// the group's size.  Returns to every active lane the counter's value before
// its group's addition plus the lane's rank in the group, i.e. its slot when
// the counter is a cursor.  Every lane of the wavefront must make the call.
__device__ __forceinline__ int32_t wave_count_add(int32_t *counter, bool active, int32_t l,
                                                  int nbits) {
    const int lane = threadIdx.x & 63;
    unsigned long long same = __ballot(active);
    for (int bit = 0; bit < nbits; ++bit) {
        const bool on = (l >> bit) & 1;
        const unsigned long long bb = __ballot(on);
        same &= on ? bb : ~bb;
    }
    const int rank = __popcll(same & ((1ull << lane) - 1ull));
    int32_t base = 0;
    if (active && rank == 0) base = atomicAdd(&counter[l], (int32_t)__popcll(same));
    const int leader = active ? __ffsll((unsigned long long)same) - 1 : lane;
    base = __shfl(base, leader, 64);
    return base + rank;
}

// Deterministic sum of one double per thread over each kAT-thread part of an
// NT-thread block (fixed tree, the same for every part and every NT); every
// thread gets its part's sum.
template <int NT = kAT>
__device__ __forceinline__ double block_sum_det(double v, double *sh) {
    static_assert(NT % kAT == 0, "block of whole parts");
    sh[threadIdx.x] = v;
    __syncthreads();
    const int b = NT == kAT ? 0 : (int)(threadIdx.x & ~(kAT - 1));
    const int i = NT == kAT ? (int)threadIdx.x : (int)(threadIdx.x & (kAT - 1));
#pragma unroll
    for (int s = kAT / 2; s > 0; s >>= 1) {
        if (i < s) sh[b + i] = sh[b + i] + sh[b + i + s];
        __syncthreads();
    }
    double r = sh[b];
    __syncthreads();
    return r;
}

template <int NT = kAT>
__device__ __forceinline__ double block_max(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Fixed point of the center sums.  Every coordinate is quantised to an
// integer q = rint(x * 2^s) with s chosen per run so that |q| <= 2^31
// (|x| <= max|x| < 2^e, s = 31 - e); the error of one coordinate is at most
// 2^-32 * 2^e <= 2^-31 max|x|, far below a float32 ulp of the mean.  The
// integers are summed exactly in int64 (no overflow below 2^32 points), so a
// sum does not depend on the order of the additions.
__device__ __forceinline__ int fix_shift_of(uint32_t absmax_bits) {
    const float m = __uint_as_float(absmax_bits);
    int e = 0;
    if (m > 0.0f) frexpf(m, &e);  // m < 2^e
    return 31 - e;
}

__device__ __forceinline__ long long to_fixed(float x, int s) {
    return (long long)(int)rintf(ldexpf(x, s));
}

// Reference point m of a run: the midpoint of its bounding box (box = ordered
// bits of the attribute minima, then maxima).
__device__ __forceinline__ float box_mid(const uint32_t *box, int d, int j) {
    return 0.5f * (ordered_float(box[j]) + ordered_float(box[d + j]));
}

}  // namespace subkm_lloyd

// ---------------------------------------------------------------------------
// Launchers of the wide-run kernels (lloyd_wide.hip).  Runs [r0, r0 + nr) of
// the device plan are contiguous and all take the wide path; their
// assignment items are items [i0, i0 + ni) and their update items
// [u0, u0 + nu).
namespace subkm_lloyd {

// Split-bfloat16 fragments and squared norms of the centers of every run in
// [r0, r0 + nr) with split set (kt_max = largest number of 16-center tiles).
subkm_status wide_split_prep(subkm_ctx *ctx, int r0, int nr, int kt_max, int steps_max,
                             const DevRun *runs, const float *C, const uint32_t *boxes,
                             uint4 *frags, float *cnorm, RunState *rs);

// Split-bfloat16 assignment of items [i0, i0 + ni) (runs of one step count S =
// ceil(d / 32), 1 <= S <= 4).
subkm_status wide_assign_split(subkm_ctx *ctx, int S, int i0, int ni, const float *P,
                               const DevRun *runs, const Item *items, const float *C,
                               const uint4 *frags, const float *cnorm, int32_t *labels,
                               RunState *rs, double *objpart, const uint32_t *boxes,
                               int last_pass);

// Exact center update of the wide runs from their labels (counted per
// center by the assignment): starts, points ordered by label, then
// per-center fixed-point sums and the run's convergence decision.
// order holds the point indices grouped by label at lab_off and their
// labels at olab_off + lab_off; gsum the int64 sums of the wide runs with
// d <= kWalkD (at sum_off, zero between calls).  Walk items [w0, w0 + nw)
// cover kWalkB * DevRun::wpp positions each.
subkm_status wide_update(subkm_ctx *ctx, int r0, int nr, int i0, int ni, int w0, int nw, int u0,
                         int nu, const float *P, const DevRun *runs, const Item *items,
                         const int32_t *labels, float *C, RunState *rs, int32_t *cnt,
                         int32_t *order, int64_t olab_off, long long *gsum, double tol);

}  // namespace subkm_lloyd
