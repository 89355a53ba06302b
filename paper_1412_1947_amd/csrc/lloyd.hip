// Lloyd's k-means for many independent runs (Sec. II Algorithm 1 step 4 in
// every subcluster; Sec. I and Sec. V for the final run on the local
// centers).
//
// Assignment (every form).  A tile of 256 points, one per thread, against the
// run's centers staged in LDS.  Every thread tracks its two smallest float32
// distances; when their gap is not larger than the rounding-error bound of
// the float32 arithmetic, the point is re-assigned with binary64 distances
// (attributes left to right, lowest center index on ties), one wavefront per
// such point.  Labels are therefore those of exact arithmetic on the float32
// inputs.  The objective uses the binary64 distance to the chosen center.
//
// Update.  Every point adds its coordinates, as 64-bit fixed point scaled by
// a per-run power of two, to its center's sum in LDS.  Integer sums are exact,
// so the new centers do not depend on the order in which threads, blocks or
// forms add them; a center without points stays.  The largest center move
// (binary64) decides convergence (strictly below tol).
//
// Forms.
//   batched  one cooperative persistent launch for all runs and all
//            iterations.  Run r is split over G_r blocks (chosen by a
//            largest-work-first schedule on the host); after every
//            assignment the G_r blocks exchange their partial sums through
//            global memory behind a per-run arrival counter, and each block
//            forms the same new centers from them in the same order.
//   plain    one run at a time: per iteration one assign+accumulate launch
//            over the run's tiles and one finalize launch.
// Runs whose k*d exceeds the LDS budget use launch-per-phase kernels for all
// runs together (assignment here or in lloyd_wide.hip, exact update through
// a label sort in lloyd_wide.hip).
#include "lloyd_dev.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <queue>
#include <tuple>
#include <type_traits>
#include <vector>

#pragma clang fp contract(off)

namespace {

using namespace subkm_lloyd;

constexpr int kCF = 4608;           // floats of centers held in LDS (fused path)
constexpr int kSumW = 4096;         // int64 center sums held in LDS (fused path)
constexpr int kMaxK = 1024;         // centers per run in the fused path
constexpr int kLdsFloats = 8192;    // centers staged per pass (scan-update path)
constexpr long long kSpinLimit = 1ll << 26;
constexpr int kMaxG = 128;         // blocks per run in the batched form
constexpr int64_t kXAtomMax = 1 << 18;  // shared-totals exchange: most atomics per move
constexpr int kExB = 16;           // exchange loads in flight per thread
constexpr int kChunkF = 8192;       // center floats staged per chunk (chunked path)
constexpr int kWideCenters = 16;    // centers per update item (wide runs)
constexpr int64_t kWalkMinBlocks = 512;  // blocks a walk launch keeps when narrow points share wavefronts
constexpr int64_t kHugeRun = 1 << 15; // points beyond which a run with moves takes the wide path
constexpr int kUList = 256;         // deferred uncertain points per block and pass (split path)

// Float32 squared distances of this thread's point against centers sC[0..nc)
// (row-major, d per row); keeps the two smallest values and the first index
// of the smallest (strict <, centers in ascending order).
template <int D>
__device__ __forceinline__ void scan_centers(const float *x, const float *xg, const float *sC,
                                             int c0, int nc, int d, float &b1, float &b2,
                                             int32_t &i1) {
    for (int c = 0; c < nc; ++c) {
        const float *cc = sC + c * d;
        float acc = 0.0f;
        if (D > 0) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                float t = x[j] - cc[j];
                acc = __builtin_fmaf(t, t, acc);
            }
        } else {
            for (int j = 0; j < d; ++j) {
                float t = xg[j] - cc[j];
                acc = __builtin_fmaf(t, t, acc);
            }
        }
        b2 = fminf(b2, fmaxf(acc, b1));
        bool lt = acc < b1;
        b1 = lt ? acc : b1;
        i1 = lt ? c0 + c : i1;
    }
}

// The gap between the two smallest float32 distances is certain iff it is
// larger than the error bound of both: |D^ - D| <= gamma_{d+2} D (one
// rounding per subtraction, one per FMA), with a safety factor of 2 and an
// absolute term for results in the subnormal range.
__device__ __forceinline__ bool certain_gap(float b1, float b2, int d, int k) {
    const float gam = 2.0f * (float)(d + 2) * 5.9604645e-8f;
    const float slack = (float)(2 * d + 2) * 2.8025969e-45f;
    return k == 1 || (b2 - b1) > gam * (b1 + b2) + slack;
}

// Binary64 re-assignment of the uncertain points of a tile (listed in
// s_list), one wavefront per point; results land in s_newlab[thread].
__device__ void recheck_tile(const float *X, int64_t first, const float *Csrc, int d, int k,
                             const int32_t *s_list, uint32_t nl, int32_t *s_newlab) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (uint32_t q = wave; q < nl; q += kAT / 64) {
        const int t = s_list[q];
        const int32_t w = wave_argmin64(X + (first + t) * d, Csrc, d, k);
        if (lane == 0) s_newlab[t] = w;
    }
}

// ---------------------------------------------------------------------------
// LDS of the fused kernels.  Centers are held row-major (c * d + j) for the
// vector path and dim-major with a padded pitch (j * (k + 16) + c) for the
// matrix-core path, whose operand reads are then free of bank conflicts.
// NT is the block size: the matrix-core persistent kernel of narrow points
// runs 512 threads (two 256-point tiles at a time) so that four wavefronts
// share each SIMD within the LDS of two blocks per CU.
template <int NT>
struct FusedLdsT {
    static constexpr int kThreads = NT;
    float sC[kCF];
    float cn[kMaxK + 16];  // matrix-core path: ||c - m||^2, +inf past k
    long long s_sum[kSumW];
    unsigned int s_cnt[kMaxK];
    int32_t s_list[kAT];   // vector path (256-thread blocks only)
    int32_t s_newlab[kAT];
    int32_t s_lab[NT];     // stage-1 label, bit 31 set when uncertain
    double s_red[NT];
    float s_R;             // matrix-core path: max_c ||c - m||
    uint32_t s_nlist;
};
using FusedLds = FusedLdsT<kAT>;

// This thread's index, opaque to the optimizer: loops of the persistent
// kernel that start at it would otherwise have their per-thread index
// arithmetic hoisted out of the pass and task loops and kept live (then
// spilled) through the whole kernel.
__device__ __forceinline__ int opaque_tid() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

template <bool MF>
__device__ __forceinline__ int cidx(int c, int j, int d, int ldk) {
    return MF ? j * ldk + c : c * d + j;
}

// Index of the sum of attribute j of center c in s_sum.  On the matrix-core
// path (D a power of two) the attributes of row c are permuted by an XOR with
// bits of c: the 64 LDS banks take 32 int64 per pass, and without the
// permutation the points of one wavefront that add attribute j to different
// centers would all land on the few banks of column j.  Every reader and
// writer of s_sum goes through this index (or works elementwise on the whole
// array), so the permutation is invisible outside the LDS.
template <int D, bool MF>
__device__ __forceinline__ int sum_idx(int c, int j, int d) {
    if constexpr (MF && D >= 4) {
        constexpr int R = D >= 32 ? 1 : 32 / D;   // rows per pass over the banks
        constexpr int M = (D >= 32 ? 32 : D) - 1;
        return c * D + (j ^ ((c / R) & M));
    } else {
        return c * d + j;
    }
}

// binary64 distance of a point (global memory) to center c held in LDS
template <bool MF>
__device__ __forceinline__ double dist64_lds(const float *x, const float *sC, int c, int d, int ldk) {
    double acc = 0.0;
    for (int j = 0; j < d; ++j) {
        double q = (double)x[j] - (double)sC[cidx<MF>(c, j, d, ldk)];
        acc = acc + q * q;
    }
    return acc;
}

template <bool MF>
__device__ int32_t wave_argmin64_lds(const float *x, const float *sC, int d, int k, int ldk) {
    const int lane = threadIdx.x & 63;
    double best = INFINITY;
    int32_t bi = 0x7fffffff;
    for (int c = lane; c < k; c += 64) {
        double v = dist64_lds<MF>(x, sC, c, d, ldk);
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

// Exact nearest center of one point x (a row in global memory) among the k
// centers held dim-major in LDS, by the whole wavefront (lanes over
// centers): the result of the binary64 argmin over all centers (attributes
// left to right, lowest index on ties), found in two steps.  Float32
// distances, each within gam = 2 (D + 2) u of the exact one (twice the
// bound of D + 2 roundings of nonnegative terms), give the minimum m; every
// center at the exact minimum distance has a float32 distance at most
// m (1 + 2 gam) (plus a margin for results in the subnormal range), and
// every center above that bound is farther than the minimum by more than
// the binary64 rounding can bridge.  Only the centers under the bound
// (usually one or two) get binary64 distances.
template <int D>
__device__ __forceinline__ int32_t wave_argmin_exact(const float *x, const float *sC, int k,
                                                  int ldk) {
    constexpr int KL = ((kCF / D - 16) + 63) / 64;  // centers per lane at most
    const int lane = threadIdx.x & 63;
    // narrow points are held in registers, wide ones read again (cached)
    constexpr bool kHold = D <= 16;
    float xs[kHold ? D : 1];
    if constexpr (kHold) {
#pragma unroll
        for (int j = 0; j < D; ++j) xs[j] = x[j];
    }
    auto xj = [&](int j) { return kHold ? xs[kHold ? j : 0] : x[j]; };
    float d32[KL];
    float m = INFINITY;
#pragma unroll
    for (int u = 0; u < KL; ++u) {
        const int c = lane + 64 * u;
        float a = INFINITY;
        if (c < k) {
            a = 0.0f;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const float t = xj(j) - sC[j * ldk + c];
                a = __builtin_fmaf(t, t, a);
            }
        }
        d32[u] = a;
        m = fminf(m, a);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fminf(m, __shfl_xor(m, o, 64));
    const float gam = 2.0f * (float)(D + 2) * 5.9604645e-8f;
    const float thr = m * (1.0f + 2.0f * gam) + (float)(4 * D + 4) * 2.8025969e-45f;
    double best = INFINITY;
    int32_t bi = 0x7fffffff;
#pragma unroll
    for (int u = 0; u < KL; ++u) {
        if (d32[u] <= thr) {  // false past k (+inf)
            const int c = lane + 64 * u;
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const double q = (double)xj(j) - (double)sC[j * ldk + c];
                acc = acc + q * q;
            }
            if (acc < best) {  // this lane's centers ascend: the first of equals stays
                best = acc;
                bi = c;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int32_t oi = __shfl_xor(bi, o, 64);
        if (ob < best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
        }
    }
    return bi;
}

// Matrix-core path: squared norms of the centered centers and their maximum.
template <int D, class LT>
__device__ void center_norms(LT &L, const uint32_t *box, int k, int ldk) {
    float mx = 0.0f;
    for (int c = threadIdx.x; c < kMaxK + 16 && c < ((k + 15) & ~15); c += LT::kThreads) {
        float a = INFINITY;
        if (c < k) {
            a = 0.0f;
#pragma unroll 4
            for (int j = 0; j < D; ++j) {
                const float t = L.sC[j * ldk + c] - box_mid(box, D, j);
                a = __builtin_fmaf(t, t, a);
            }
            mx = fmaxf(mx, a);
        }
        L.cn[c] = a;
    }
    const double r = block_max<LT::kThreads>((double)mx, L.s_red);
    if (threadIdx.x == 0) L.s_R = sqrtf((float)r);
    __syncthreads();
}

// Stage 1 on matrix cores (v_mfma_f32_16x16x4_f32).  A wavefront takes 64
// points as four groups of 16; a 16x16 output tile holds the dot products of
// 16 centers (rows) with 16 points (columns): lane l sees point l % 16 of a
// group and centers 4 * (l / 16) + r, r = 0..3, of the tile.  Both sides are
// centered on m; v = ||c - m||^2 - 2 (x - m).(c - m) ranks the centers like
// ||x - c||^2 (the accumulator starts at ||c - m||^2).  Every lane keeps the two smallest v of its centers; four
// lanes share a point and merge at the end.  The gap of the two smallest is
// certain when it exceeds twice the error bound
//     E = 2 (d + 5) u (||x - m|| + max_c ||c - m||)^2,   u = 2^-24,
// which covers the rounding of the centering, the products, the sums and the
// final combination (with a factor 2 of margin).  Results go to L.s_lab.
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Raw coordinates of a tile as the matrix-core lanes hold them: lane
// (col = l % 16, kk = l / 16) of a wavefront holds attributes kk + 4 q of
// point col of each of its four 16-point groups.  Loads are unconditional
// (rows past n are clamped to the last row; their values are never used),
// so all of them are in flight together.
template <int D>
__device__ __forceinline__ void load_tile(const float *X, int64_t first_w, int64_t n,
                                          float (&xr)[4][D / 4]) {
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, kk = lane >> 4;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        int64_t p = first_w + g * 16 + col;
        p = p < n ? p : n - 1;
#pragma unroll
        for (int q = 0; q < D / 4; ++q) xr[g][q] = X[p * D + kk + 4 * q];
    }
}

// The tile centered on the box midpoint m (points past n become 0) and the
// norms ||x - m|| of its points, as the matrix-core lanes hold them.  The raw
// registers are free afterwards (the next tile can be loaded into them).
template <int D>
__device__ __forceinline__ void center_tile(const float (&xr)[4][D / 4], const uint32_t *box,
                                            int64_t first_w, int64_t n, float (&xb)[4][D / 4],
                                            float (&xn)[4]) {
    constexpr int KQ = D / 4;
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, kk = lane >> 4;
    float mq[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) mq[q] = box_mid(box, D, kk + 4 * q);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const bool ok = first_w + g * 16 + col < n;
        float s2 = 0.0f;
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            const float v = ok ? xr[g][q] - mq[q] : 0.0f;
            xb[g][q] = v;
            s2 = __builtin_fmaf(v, v, s2);
        }
        s2 += lane_xor16(s2);
        s2 += lane_xor32(s2);
        xn[g] = sqrtf(s2);
    }
}

// Stage 1 of a centered tile (xb, xn from center_tile).  Certain points are
// added to the sums from their raw coordinates, read again from X (the tile
// was just loaded, so the reads hit the caches), which keeps the raw tile out
// of the registers while the products run.
template <int D, class LT>
__device__ void stage1_mfma(LT &L, const float (&xb)[4][D / 4], const float (&xn)[4],
                            const float *X, int64_t first_w, int64_t n, int k, int ldk,
                            const uint32_t *box, int32_t *lab_out, bool accumulate, int shift,
                            int32_t *wlab) {
    constexpr int KQ = D / 4;
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, kk = lane >> 4;
    float mq[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) mq[q] = box_mid(box, D, kk + 4 * q);
    float b1[4], b2[4];
    int32_t i1[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        b1[g] = INFINITY;
        b2[g] = INFINITY;
        i1[g] = 0;
    }
    // The products of a block of 16 centers: the bias ||c - m||^2 of the
    // lane's four output rows (centers c0 + 4 kk + r) starts the
    // accumulator; the centers are scaled by -2 (exact), so the accumulator
    // ends as v itself.  Rows of sC are padded to k + 16 and cn holds +inf
    // up to the next multiple of 16, so every read stays inside the arrays;
    // centers past k are zeroed by a bit mask (the loads stay unconditional,
    // with no branch and wait each) and their values are never selected.
    auto products = [&](int c0, floatx4 (&acc)[4]) {
        const int cA = c0 + col;
        const uint32_t vmask = cA < k ? 0xFFFFFFFFu : 0u;
        float ca[KQ];
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            const float cv = L.sC[(kk + 4 * q) * ldk + cA];
            ca[q] = __uint_as_float(__float_as_uint(-2.0f * (cv - mq[q])) & vmask);
        }
        const floatx4 cinit = {L.cn[c0 + 4 * kk], L.cn[c0 + 4 * kk + 1], L.cn[c0 + 4 * kk + 2],
                               L.cn[c0 + 4 * kk + 3]};
#pragma unroll
        for (int g = 0; g < 4; ++g) acc[g] = cinit;
#pragma unroll
        for (int q = 0; q < KQ; ++q)
#pragma unroll
            for (int g = 0; g < 4; ++g) acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[q], xb[g][q], acc[g], 0, 0, 0);
    };
    // The two smallest values of each point's four lanes and the first
    // index of the smallest, centers in ascending order (strict <).
    auto select = [&](int c0, const floatx4 (&acc)[4]) {
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float v = acc[g][r];
                // b1 <= b2 always holds, so the new second-smallest is the median
                b2[g] = __builtin_amdgcn_fmed3f(v, b1[g], b2[g]);
                const bool lt = v < b1[g];
                b1[g] = lt ? v : b1[g];
                i1[g] = lt ? c0 + 4 * kk + r : i1[g];
            }
    };
    for (int c0 = 0; c0 < k; c0 += 16) {
        floatx4 acc[4];
        products(c0, acc);
        select(c0, acc);
    }
    const float Rc = L.s_R;
    const float Ku = 2.0f * (float)(D + 5) * 5.9604645e-8f;
    // raw attributes for the sums, loaded before the merge (rows past n
    // clamped) for narrow points; wide ones load at the addition
    constexpr bool kEarly = D <= 16;
    float xv[4][KQ];
    if (kEarly && accumulate) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            int64_t p = first_w + g * 16 + col;
            p = p < n ? p : n - 1;
            const float *xp = X + p * D + kk;
#pragma unroll
            for (int q = 0; q < KQ; ++q) xv[g][q] = xp[4 * q];
        }
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
        for (int o = 16; o <= 32; o <<= 1) {
            const float ob1 = o == 16 ? lane_xor16(b1[g]) : lane_xor32(b1[g]);
            const float ob2 = o == 16 ? lane_xor16(b2[g]) : lane_xor32(b2[g]);
            const int32_t oi = o == 16 ? lane_xor16(i1[g]) : lane_xor32(i1[g]);
            const float nb2 = fminf(fminf(b2[g], ob2), fmaxf(b1[g], ob1));
            const bool take = (ob1 < b1[g]) | ((ob1 == b1[g]) & (oi < i1[g]));  // no branch
            b1[g] = take ? ob1 : b1[g];
            i1[g] = take ? oi : i1[g];
            b2[g] = nb2;
        }
        // the four lanes of a point now agree on (b1, b2, i1)
        const int64_t p = first_w + g * 16 + col;
        const float s = xn[g] + Rc;
        const float E = Ku * s * s + 1e-30f;
        const bool certain = k == 1 || (b2[g] - b1[g]) > 2.0f * E;
        if (p < n && certain) {
            // a certain point is labelled and added to its center right here,
            // from the registers that hold it (each lane its KQ attributes)
            if (kk == 0) lab_out[p] = i1[g];
            if (accumulate) {
                if (kk == 0) atomicAdd(&L.s_cnt[i1[g]], 1u);
                if constexpr (!kEarly) {
                    const float *xp = X + p * D + kk;
#pragma unroll
                    for (int q = 0; q < KQ; ++q) xv[g][q] = xp[4 * q];
                }
#pragma unroll
                for (int q = 0; q < KQ; ++q)
                    atomicAdd((unsigned long long *)&L.s_sum[sum_idx<D, true>(i1[g], kk + 4 * q, D)],
                              (unsigned long long)to_fixed(xv[g][q], shift));
            }
        }
        if (kk == 0) wlab[g * 16 + col] = i1[g] | (certain ? 0 : (int32_t)0x80000000);
    }
}

// Matrix-core tile of one wavefront (64 points, first_w .. first_w + 63):
// stage 1 labels (and, if asked, accumulates) every point whose nearest center
// is certain; the uncertain ones are re-assigned in binary64 by the whole
// wavefront, one after the other, then labelled and accumulated by their own
// lane.  No block barrier: only the wavefront's own LDS slice is exchanged.
// On the final pass (no accumulation) every lane returns the binary64
// objective of its point.
// Second half of a matrix-core tile, after stage 1 has filled wlab.
// With DEFER, on a pass with an update, the uncertain points go to the
// block's list (resolve_deferred takes them before the exchange) as long as
// it has room; the others, and all of them on the last pass (whose per-tile
// objective needs the labels now), are re-assigned here.
template <int D, bool DEFER = false, class LT>
__device__ double wave_tile_finish(LT &L, const float *X, int64_t first_w, int64_t n, int k, int ldk,
                                   int32_t *lab_out, bool accumulate, int shift,
                                   unsigned long long &nrecheck, const int32_t *wlab) {
    const int lane = threadIdx.x & 63;
    const int64_t i = first_w + lane;
    const bool valid = i < n;
    const float *xg = X + (valid ? i : 0) * D;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int32_t sl = wlab[lane];
    int32_t i1 = sl & 0x7fffffff;
    unsigned long long todo = __ballot(valid && sl < 0);
    nrecheck += (unsigned long long)__popcll(todo);
    if constexpr (DEFER) {
        if (accumulate && todo) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&L.s_nu, (uint32_t)__popcll(todo));
            base = (uint32_t)__builtin_amdgcn_readlane((int)base, 0);
            const bool mine = (todo >> lane) & 1ull;
            const uint32_t slot = base + (uint32_t)__popcll(todo & ((1ull << lane) - 1ull));
            if (mine && slot < (uint32_t)kUList) L.s_ulist[slot] = (int32_t)i;
            todo = __ballot(mine && slot >= (uint32_t)kUList);
        }
    }
    while (todo) {
        const int t = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const int32_t w = wave_argmin_exact<D>(X + (first_w + t) * D, L.sC, k, ldk);
        if (lane == t) {
            i1 = w;
            lab_out[i] = w;
            if (accumulate) {
                atomicAdd(&L.s_cnt[w], 1u);
                for (int j = 0; j < D; ++j)
                    atomicAdd((unsigned long long *)&L.s_sum[sum_idx<D, true>(w, j, D)],
                              (unsigned long long)to_fixed(xg[j], shift));
            }
        }
    }
    double obj = 0.0;
    if (valid && !accumulate) obj = dist64_lds<true>(xg, L.sC, i1, D, ldk);
    return obj;
}

template <int D, class LT>
__device__ double wave_tile_mf(LT &L, const float (&xb)[4][D / 4], const float (&xn)[4],
                               const float *X, int64_t first_w, int64_t n, int k, int ldk,
                               const uint32_t *box, int32_t *lab_out, bool accumulate, int shift,
                               unsigned long long &nrecheck) {
    int32_t *wlab = L.s_lab + (threadIdx.x >> 6) * 64;
    stage1_mfma<D>(L, xb, xn, X, first_w, n, k, ldk, box, lab_out, accumulate, shift, wlab);
    return wave_tile_finish<D>(L, X, first_w, n, k, ldk, lab_out, accumulate, shift, nrecheck, wlab);
}

// ---------------------------------------------------------------------------
// Matrix-core path on split bfloat16 (D = 8, 16, 32).  The float32 matrix
// instruction (16x16x4) keeps the SIMD busy for 32 cycles and does not overlap
// the selection that follows on the same SIMD, so stage 1 runs on
// v_mfma_f32_16x16x32_bf16 instead: both centered operands are split into two
// bfloat16 parts (round to nearest), a = ah + al and -2 c = ch + cl, and the
// four products ch ah, cl ah, ch al, cl al, each exact in float32, are summed
// by the instruction with K laid out as four terms of D attributes
// (kappa = term * D + j).  The accumulator starts at ||c - m||^2 + Q, with Q
// at least the largest ||x - m||^2 of the run's box, so every value is
// positive.  Error bound of one value v, s = ||x - m|| + R, u = 2^-24:
//   split residuals        4 * 2^-16 sum_j |a_j| |c_j|  <=  2^-16 s^2
//   centering and norms    (D + 3) u (s^2 + Q)
//   accumulation           (4 D + 1) additions that may each round toward
//                          zero, on partial sums below 1.03 (s^2 + Q):
//                          2 (4 D + 1) u (1.03 (s^2 + Q))
// so E = 2^-16 s^2 + (D + 3 + 2.06 (4 D + 1)) u (s^2 + Q) + 1e-30, and the
// gap of the two smallest values is certain when it exceeds 2 E (plus the
// bits the selection keys drop, see stage1_bf).  Uncertain points are
// checked again on float32 matrix cores and, if still close, in binary64
// (resolve_deferred, wave_argmin_exact), so labels are those of the other
// paths.
template <int D>
constexpr bool kBF = D == 8 || D == 16 || D == 32;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kBfMaxK = kCF / 8 - 16;  // centers of a split-path run (D >= 8)

template <int NT>
struct BfLdsT {
    static constexpr int kThreads = NT;
    float sC[kCF];           // centers, dim-major with pitch k + 16 (as the float32 path)
    bf16x8 sA[kCF / 4];      // split -2 (c - m): per center D/4 chunks of 8 (ch chunks, then cl)
    float cn[kBfMaxK + 16];  // ||c - m||^2, +inf past k
    long long s_sum[kSumW];
    unsigned int s_cnt[kBfMaxK];
    int32_t s_lab[NT];
    double s_red[NT];
    int32_t s_ulist[kUList];  // uncertain points of this pass, resolved before the exchange
    uint32_t s_nu;
    uint32_t s_next;          // next 64-point piece of the block's tiles (passes with an update)
    float s_mid[32];          // the run's box midpoint m (read here, not held in registers)
    float s_Q;                // offset that makes every value positive (see stage1_bf)
    float s_R;
};

// Chunk q of center c in sA.  A wavefront reads chunk q of 16 consecutive
// centers in one instruction; chunk q of center c sits at position q ^ f(c)
// of its row so that those 16 reads cover the 64 banks once.
template <int D>
__device__ __forceinline__ int sa_idx(int c, int q) {
    constexpr int NQ = D / 4;   // chunks per center
    constexpr int RP = 64 / D;  // centers per 256 bytes
    return c * NQ + (q ^ ((c / RP) & (NQ - 1)));
}

// Norms, maximum norm and split operands of the run's centers (after every
// update).  Centers k .. 16 ceil(k / 16) - 1 get zero operands and an
// infinite norm, so their values are +inf and never selected.
template <int D, class LT>
__device__ void center_prep_bf(LT &L, const uint32_t *box, int k, int ldk) {
    float mx = 0.0f;
    const int kr = (k + 15) & ~15;
    for (int c = opaque_tid(); c < kr; c += LT::kThreads) {
        float a = INFINITY;
        if (c < k) {
            a = 0.0f;
#pragma unroll
            for (int q = 0; q < D / 8; ++q) {
                bf16x8 hi, lo;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int j = 8 * q + e;
                    const float t = L.sC[j * ldk + c] - L.s_mid[j];
                    a = __builtin_fmaf(t, t, a);
                    const float v = -2.0f * t;
                    const __bf16 h = (__bf16)v;
                    hi[e] = h;
                    lo[e] = (__bf16)(v - (float)h);
                }
                L.sA[sa_idx<D>(c, q)] = hi;
                L.sA[sa_idx<D>(c, D / 8 + q)] = lo;
            }
            mx = fmaxf(mx, a);
        } else {
            const bf16x8 z = {};
#pragma unroll
            for (int q = 0; q < D / 4; ++q) L.sA[sa_idx<D>(c, q)] = z;
        }
        L.cn[c] = a + L.s_Q;  // +inf past k
    }
    const double r = block_max<LT::kThreads>((double)mx, L.s_red);
    if (threadIdx.x == 0) L.s_R = sqrtf((float)r);
    __syncthreads();
}

// Raw attributes of a tile as the split path's lanes use them: lane
// (col = l % 16, kg = l / 16) holds attributes j0 .. j0 + 7, j0 = 8 kg mod D,
// of point col of each 16-point group (rows past n clamped to the last).
template <int D>
__device__ __forceinline__ void load_tile_bf(const float *X, int64_t first_w, int64_t n,
                                             float (&xr)[4][8]) {
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, kg = lane >> 4;
    const int j0 = (8 * kg) % D;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        int64_t p = first_w + g * 16 + col;
        p = p < n ? p : n - 1;
        const float4 *src = reinterpret_cast<const float4 *>(X + p * D + j0);
        const float4 u = src[0], w = src[1];
        xr[g][0] = u.x; xr[g][1] = u.y; xr[g][2] = u.z; xr[g][3] = u.w;
        xr[g][4] = w.x; xr[g][5] = w.y; xr[g][6] = w.z; xr[g][7] = w.w;
    }
}

// Centered and split tile (points past n become 0), the norms ||x - m||, and
// the raw attributes this lane adds to the sums (xa): the 32 / D lanes that
// hold the same 8 attributes of a point take D / 4 of them each, lane kg the
// part (8 kg / D), so that only those stay in registers through stage 1.
template <int D>
__device__ __forceinline__ void split_tile_bf(const float (&xr)[4][8], const float *s_mid,
                                              int64_t first_w, int64_t n, bf16x8 (&ah)[4],
                                              bf16x8 (&al)[4], float (&xn)[4],
                                              float (&xa)[4][D / 4]) {
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, kg = lane >> 4;
    const int j0 = (8 * kg) % D;
    float mq[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) mq[e] = s_mid[j0 + e];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const bool ok = first_w + g * 16 + col < n;
        float s2 = 0.0f;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float a = ok ? xr[g][e] - mq[e] : 0.0f;
            s2 = __builtin_fmaf(a, a, s2);
            const __bf16 h = (__bf16)a;
            ah[g][e] = h;
            al[g][e] = (__bf16)(a - (float)h);
        }
        // the lanes that hold the point's other attributes
        if constexpr (D >= 16) s2 += lane_xor16(s2);
        if constexpr (D >= 32) s2 += lane_xor32(s2);
        xn[g] = sqrtf(s2);
        constexpr int QA = D / 4;
        const int part = (8 * kg) / D;
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            // element part * QA + q, chosen without indexing registers
            float v = xr[g][q];
#pragma unroll
            for (int pp = 1; pp < 8 / QA; ++pp) v = part == pp ? xr[g][pp * QA + q] : v;
            xa[g][q] = v;
        }
    }
}

// Stage 1 of a split tile: labels and (if asked) sums of the certain points,
// stage-1 labels with the uncertain flag in wlab, as stage1_mfma.  Each lane
// adds its share xa of its point's attributes (from split_tile_bf).  Once
// the products are done, the next tile's raw attributes are requested into
// xq (next_w < 0: none), so that their loads overlap the rest of the tile.
template <int D, class LT>
__device__ void stage1_bf(LT &L, const bf16x8 (&ah)[4], const bf16x8 (&al)[4], const float (&xn)[4],
                          const float (&xa)[4][D / 4], float (&xq)[4][8], int64_t next_w, const float *X,
                          int64_t first_w, int64_t n, int k, int32_t *lab_out, bool accumulate,
                          int shift, int32_t *wlab) {
    constexpr int S = D / 8;                 // instructions per group and center block
    constexpr int NA = D >= 16 ? D / 16 : 1;  // distinct A operands per lane
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, kg = lane >> 4;
    // A operand of instruction s: chunk (t & 1) D/8 + j0/8 of the center,
    // t = (32 s + 8 kg) / D the term; terms 2 and 3 repeat the chunks of 0 and 1
    int qa[NA];
#pragma unroll
    for (int s = 0; s < NA; ++s) {
        const int t = (32 * s + 8 * kg) / D, j0 = (32 * s + 8 * kg) % D;
        qa[s] = (t & 1) * (D / 8) + j0 / 8;
    }
    // B operand: al for terms 2 and 3 (a lane-dependent choice only for D = 8)
    bf16x8 b8[4];
    if constexpr (D == 8) {
#pragma unroll
        for (int g = 0; g < 4; ++g) b8[g] = kg >= 2 ? al[g] : ah[g];
    }
    // Selection on keys: every value is positive (the accumulator starts at
    // ||c - m||^2 + Q, Q >= max ||x - m||^2, and the error bound is far below
    // Q / 256), so its bits order like the value as unsigned integers.  The
    // low IB bits are replaced by the lane's candidate number (c0 / 4 + r),
    // which makes one minimum and one median per value keep the two smallest
    // keys and the first one's center; the bits dropped are covered in the
    // certainty test below.
    const int nlocal = 4 * ((k + 15) >> 4);         // candidates per lane
    const int IB = 32 - __builtin_clz((unsigned)(nlocal - 1));
    const uint32_t kmask = (1u << IB) - 1u;
    uint32_t k1[4], k2[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        k1[g] = 0xFFFFFFFFu;
        k2[g] = 0xFFFFFFFFu;
    }
    for (int c0 = 0; c0 < k; c0 += 16) {
        bf16x8 A[NA];
#pragma unroll
        for (int s = 0; s < NA; ++s) A[s] = L.sA[sa_idx<D>(c0 + col, qa[s])];
        const floatx4 cinit = {L.cn[c0 + 4 * kg], L.cn[c0 + 4 * kg + 1], L.cn[c0 + 4 * kg + 2],
                               L.cn[c0 + 4 * kg + 3]};
        floatx4 acc[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            acc[g] = cinit;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const bf16x8 B = D == 8 ? b8[g] : ((32 * s) / D >= 2 ? al[g] : ah[g]);
                acc[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[s % NA], B, acc[g], 0, 0, 0);
            }
        }
        const uint32_t base = (uint32_t)(c0 >> 2);
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t bits = __float_as_uint(acc[g][r]);
                const uint32_t key = bits ^ ((bits ^ (base + (uint32_t)r)) & kmask);
                // the median of (key, k1, k2) is the new second key (k1 <= k2)
                k2[g] = max(min(key, k1[g]), min(max(key, k1[g]), k2[g]));
                k1[g] = min(k1[g], key);
            }
    }
    if (next_w >= 0) load_tile_bf<D>(X, next_w, n, xq);
    // back to values (low bits cleared: at most 2^IB ulp below the value)
    // and center numbers
    float b1[4], b2[4];
    int32_t i1[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        b1[g] = __uint_as_float(k1[g] & ~kmask);
        b2[g] = __uint_as_float(k2[g] & ~kmask);
        const uint32_t l = k1[g] & kmask;
        i1[g] = (int32_t)(16 * (l >> 2) + 4 * (uint32_t)kg + (l & 3u));
    }
    const float Rc = L.s_R, Qc = L.s_Q;
    // E = Ks s^2 + Ka (s^2 + Q): the split residuals, and the centering,
    // norms and accumulation, whose terms now reach s^2 + Q
    constexpr float Ks = 1.52587890625e-05f;
    constexpr float Ka = (float)(D + 3 + 2.06 * (4 * D + 1)) * 5.9604645e-8f;
    // the dropped low bits: the smallest key's value lies at most 2^IB ulp
    // above its decoded value b1 <= b2, i.e. below 2^(IB - 23) b2 (taken twice)
    const float Kt = __uint_as_float((uint32_t)(127 + IB - 22) << 23);
    // this lane's share of its 8 attributes (see split_tile_bf)
    constexpr int QA = D / 4;
    const int part = (8 * kg) / D;
    const int j0 = (8 * kg) % D;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
        for (int o = 16; o <= 32; o <<= 1) {
            const float ob1 = o == 16 ? lane_xor16(b1[g]) : lane_xor32(b1[g]);
            const float ob2 = o == 16 ? lane_xor16(b2[g]) : lane_xor32(b2[g]);
            const int32_t oi = o == 16 ? lane_xor16(i1[g]) : lane_xor32(i1[g]);
            const float nb2 = fminf(fminf(b2[g], ob2), fmaxf(b1[g], ob1));
            const bool take = (ob1 < b1[g]) | ((ob1 == b1[g]) & (oi < i1[g]));  // no branch
            b1[g] = take ? ob1 : b1[g];
            i1[g] = take ? oi : i1[g];
            b2[g] = nb2;
        }
        const int64_t p = first_w + g * 16 + col;
        const float sx = xn[g] + Rc;
        const float s2 = sx * sx, s2q = s2 + Qc;
        const float E = Ks * s2 + Ka * s2q + 1e-30f;
        const bool certain = k == 1 || (b2[g] - b1[g]) > 2.0f * E + Kt * b2[g];
        if (p < n && certain) {
            if (kg == 0) lab_out[p] = i1[g];
            if (accumulate) {
                if (kg == 0) atomicAdd(&L.s_cnt[i1[g]], 1u);
#pragma unroll
                for (int q = 0; q < QA; ++q)
                    atomicAdd((unsigned long long *)&L.s_sum[sum_idx<D, true>(i1[g], j0 + part * QA + q, D)],
                              (unsigned long long)to_fixed(xa[g][q], shift));
            }
        }
        if (kg == 0) wlab[g * 16 + col] = i1[g] | (certain ? 0 : (int32_t)0x80000000);
    }
}

// Split-path tile of one wavefront: stage 1 on split bfloat16, then the
// binary64 re-assignment of the uncertain points and the objective.
template <int D, class LT>
__device__ double wave_tile_bf(LT &L, const bf16x8 (&ah)[4], const bf16x8 (&al)[4],
                               const float (&xn)[4], const float (&xa)[4][D / 4], float (&xq)[4][8],
                               int64_t next_w, const float *X, int64_t first_w, int64_t n, int k,
                               int ldk, int32_t *lab_out, bool accumulate, int shift,
                               unsigned long long &nrecheck) {
    int32_t *wlab = L.s_lab + (threadIdx.x >> 6) * 64;
    stage1_bf<D>(L, ah, al, xn, xa, xq, next_w, X, first_w, n, k, lab_out, accumulate, shift, wlab);
    return wave_tile_finish<D, true>(L, X, first_w, n, k, ldk, lab_out, accumulate, shift, nrecheck, wlab);
}

// The deferred uncertain points of a pass, 16 per wavefront at a time, on
// the float32 matrix cores (the products of stage1_mfma for one 16-point
// group, bound 2 (D + 5) u s^2: about a tenth of the split path's).  The
// certain ones are labelled and added to the sums; the others get the exact
// argmin.  Every thread of the block calls this after the pass's tiles.
template <int D, class LT>
__device__ void resolve_deferred(LT &L, const float *X, int k, int ldk, const uint32_t *box,
                                 int32_t *lab_out, int shift) {
    constexpr int KQ = D / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kk = lane >> 4;
    const int nu = min((int)L.s_nu, kUList);
    float mq[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) mq[q] = L.s_mid[kk + 4 * q];
    const float Rc = L.s_R;
    const float Ku = 2.0f * (float)(D + 5) * 5.9604645e-8f;
    for (int g0 = wave * 16; g0 < nu; g0 += (LT::kThreads / 64) * 16) {
        const bool ok = g0 + col < nu;
        const int32_t p = L.s_ulist[ok ? g0 + col : g0];  // a listed row either way
        float xr[KQ], xb[KQ];
#pragma unroll
        for (int q = 0; q < KQ; ++q) xr[q] = X[(int64_t)p * D + kk + 4 * q];
        float s2 = 0.0f;
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            xb[q] = xr[q] - mq[q];
            s2 = __builtin_fmaf(xb[q], xb[q], s2);
        }
        s2 += lane_xor16(s2);
        s2 += lane_xor32(s2);
        const float xn = sqrtf(s2);
        float b1 = INFINITY, b2 = INFINITY;
        int32_t i1 = 0;
        for (int c0 = 0; c0 < k; c0 += 16) {
            const int cA = c0 + col;
            const uint32_t vmask = cA < k ? 0xFFFFFFFFu : 0u;
            float ca[KQ];
#pragma unroll
            for (int q = 0; q < KQ; ++q) {
                const float cv = L.sC[(kk + 4 * q) * ldk + cA];
                ca[q] = __uint_as_float(__float_as_uint(-2.0f * (cv - mq[q])) & vmask);
            }
            floatx4 acc = {L.cn[c0 + 4 * kk], L.cn[c0 + 4 * kk + 1], L.cn[c0 + 4 * kk + 2],
                           L.cn[c0 + 4 * kk + 3]};
#pragma unroll
            for (int q = 0; q < KQ; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[q], xb[q], acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float v = acc[r];
                b2 = __builtin_amdgcn_fmed3f(v, b1, b2);
                const bool lt = v < b1;
                b1 = lt ? v : b1;
                i1 = lt ? c0 + 4 * kk + r : i1;
            }
        }
#pragma unroll
        for (int o = 16; o <= 32; o <<= 1) {
            const float ob1 = o == 16 ? lane_xor16(b1) : lane_xor32(b1);
            const float ob2 = o == 16 ? lane_xor16(b2) : lane_xor32(b2);
            const int32_t oi = o == 16 ? lane_xor16(i1) : lane_xor32(i1);
            const float nb2 = fminf(fminf(b2, ob2), fmaxf(b1, ob1));
            const bool take = (ob1 < b1) | ((ob1 == b1) & (oi < i1));
            b1 = take ? ob1 : b1;
            i1 = take ? oi : i1;
            b2 = nb2;
        }
        const float sx = xn + Rc;
        const float E = Ku * (sx * sx + L.s_Q) + 1e-30f;  // values carry the offset Q
        const bool certain = k == 1 || (b2 - b1) > 2.0f * E;
        if (ok && certain) {
            if (kk == 0) {
                lab_out[p] = i1;
                atomicAdd(&L.s_cnt[i1], 1u);
            }
#pragma unroll
            for (int q = 0; q < KQ; ++q)
                atomicAdd((unsigned long long *)&L.s_sum[sum_idx<D, true>(i1, kk + 4 * q, D)],
                          (unsigned long long)to_fixed(xr[q], shift));
        }
        unsigned long long todo = __ballot(ok && !certain && kk == 0);
        while (todo) {
            const int t = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int32_t pt = L.s_ulist[g0 + t];
            const int32_t w = wave_argmin_exact<D>(X + (int64_t)pt * D, L.sC, k, ldk);
            if (lane == 0) {
                lab_out[pt] = w;
                atomicAdd(&L.s_cnt[w], 1u);
            }
            for (int j = lane; j < D; j += 64)
                atomicAdd((unsigned long long *)&L.s_sum[sum_idx<D, true>(w, j, D)],
                          (unsigned long long)to_fixed(X[(int64_t)pt * D + j], shift));
        }
    }
}

// Assign one tile of up to 256 points of a run against all k centers held in
// LDS; optionally add the points to the fixed-point sums.  Returns the
// binary64 objective contribution of this thread's point (0 if none).
template <int D, bool MF>
__device__ __forceinline__ double fused_tile(FusedLds &L, const float *X, int64_t first, int64_t n, int d, int k,
                             int ldk, const uint32_t *box, int32_t *lab_out, bool accumulate,
                             int shift, unsigned long long *rechecks) {
    const int64_t i = first + threadIdx.x;
    const bool valid = i < n;
    const float *xg = X + (valid ? i : 0) * d;
    __syncthreads();  // the previous tile is done with the LDS lists
    if (threadIdx.x == 0) L.s_nlist = 0;
    int32_t i1;
    bool certain;
    {
        float x[D > 0 ? D : 1];
        if (D > 0) {
#pragma unroll
            for (int j = 0; j < D; ++j) x[j] = xg[j];
        }
        __syncthreads();
        float b1 = INFINITY, b2 = INFINITY;
        i1 = 0;
        scan_centers<D>(x, xg, L.sC, 0, k, d, b1, b2, i1);
        certain = certain_gap(b1, b2, d, k);
    }
    if (valid && !certain) L.s_list[atomicAdd(&L.s_nlist, 1u)] = threadIdx.x;
    __syncthreads();
    const uint32_t nl = L.s_nlist;
    if (nl) {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (uint32_t q = wave; q < nl; q += kAT / 64) {
            const int t = L.s_list[q];
            const int32_t w = wave_argmin64_lds<MF>(X + (first + t) * d, L.sC, d, k, ldk);
            if (lane == 0) L.s_newlab[t] = w;
        }
        __syncthreads();
        if (valid && !certain) i1 = L.s_newlab[threadIdx.x];
        if (threadIdx.x == 0) atomicAdd(rechecks, (unsigned long long)nl);
    }
    double obj = 0.0;
    if (valid) {
        lab_out[i] = i1;
        if (!accumulate) obj = dist64_lds<MF>(xg, L.sC, i1, d, ldk);
        if (accumulate) {
            atomicAdd(&L.s_cnt[i1], 1u);
            long long *row = L.s_sum + i1 * d;
            // lanes start at different attributes, so that one LDS atomic
            // instruction does not send all lanes to the same bank
            int j = threadIdx.x % d;
            for (int q = 0; q < d; ++q) {
                atomicAdd((unsigned long long *)&row[j], (unsigned long long)to_fixed(xg[j], shift));
                j = j + 1 == d ? 0 : j + 1;
            }
        }
    }
    return obj;
}

// New centers from the sums in L.s_sum / L.s_cnt: writes L.sC (and Cglob,
// row-major, if non-null) and returns the largest binary64 center move.
template <int D, bool MF, class LT>
__device__ double centers_from_sums(LT &L, int d, int k, int ldk, int shift, float *Cglob) {
    double mx = 0.0;
    for (int c = opaque_tid(); c < k; c += LT::kThreads) {
        const unsigned int cnt = L.s_cnt[c];
        double mv2 = 0.0;
        int j = c % d;  // rotated start: neighbouring lanes read different banks
        for (int q = 0; q < d; ++q, j = j + 1 == d ? 0 : j + 1) {
            const int e = cidx<MF>(c, j, d, ldk);
            const float old = L.sC[e];
            const double nv =
                cnt ? ldexp((double)L.s_sum[sum_idx<D, MF>(c, j, d)], -shift) / (double)cnt : (double)old;
            const double dv = nv - (double)old;
            mv2 = mv2 + dv * dv;
            const float f = (float)nv;
            L.sC[e] = f;
            if (Cglob) Cglob[c * d + j] = f;
        }
        mx = fmax(mx, sqrt(mv2));
    }
    return block_max<LT::kThreads>(mx, L.s_red);
}

// load the run's centers (row-major in global memory) into LDS
template <bool MF, class LT>
__device__ void load_centers(LT &L, const float *Cr, int d, int k, int ldk) {
    for (int e = threadIdx.x; e < k * d; e += LT::kThreads) {
        const int c = e / d, j = e - c * d;
        L.sC[cidx<MF>(c, j, d, ldk)] = Cr[e];
    }
}

// ---------------------------------------------------------------------------
// Batched form: persistent, cooperative.  Block b works through its tasks
// task_off[b] .. task_off[b+1]-1 in order; every task is one part of a run.
// A block of NT threads takes NT / 256 tiles of 256 points at a time, one
// per 256-thread part.
template <int D, bool MF, bool BF, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT > kAT ? 4 : (D > 0 && D <= 32 ? 2 : 1)))) void k_lloyd_persist(
    const float *__restrict__ P, const DevRun *__restrict__ runs, const Task *__restrict__ tasks,
    const int32_t *__restrict__ task_off, float *C, int32_t *labels, RunState *rstate,
    long long *parts, double *objpart, const uint32_t *__restrict__ boxes, int max_iter,
    double tol, int *err) {
    static_assert(MF || NT == kAT, "the vector path runs 256-thread blocks");
    static_assert(!BF || (MF && kBF<D>), "split path: matrix cores, D = 8, 16 or 32");
    using LT = std::conditional_t<BF, BfLdsT<NT>, FusedLdsT<NT>>;
    __shared__ LT L;
    for (int ti = task_off[blockIdx.x]; ti < task_off[blockIdx.x + 1]; ++ti) {
        const Task tk = tasks[ti];
        const DevRun R = runs[tk.run];
        RunState *rs = rstate + tk.run;
        const int d = D > 0 ? D : R.d;
        const int k = R.k;
        const int kd = k * d;
        const int ldk = k + 16;
        const int G = R.G;
        const int shift = fix_shift_of(rs->absmax_bits);
        const uint32_t *box = boxes + R.box_off;
        // the run's points are split over its G blocks in whole tiles
        const int64_t tiles = (R.n + kAT - 1) / kAT;
        const int64_t t0 = tiles * tk.g / G, t1 = tiles * (tk.g + 1) / G;
        const float *X = P + R.x_off;
        int32_t *lab = labels + R.lab_off;
        float *Cr = C + R.c_off;
        __syncthreads();
        load_centers<MF>(L, Cr, d, k, ldk);
        if constexpr (BF) {
            for (int j = threadIdx.x; j < D; j += NT) L.s_mid[j] = box_mid(box, D, j);
            if (threadIdx.x == 0) {
                // Q >= max ||x - m||^2 over the box, with margins: every |x_j - m_j|
                // is at most max(hi_j - m_j, m_j - lo_j), and the centered values
                // round up by a relative 2^-24 at most
                float q = 0.0f;
                for (int j = 0; j < D; ++j) {
                    const float lo = ordered_float(box[j]), hi = ordered_float(box[D + j]);
                    const float m = box_mid(box, D, j);
                    const float a = fmaxf(hi - m, m - lo) * (1.0f + 0x1p-20f);
                    q = __builtin_fmaf(a, a, q);
                }
                L.s_Q = q * (1.0f + 0x1p-8f) + 0x1p-100f;
            }
        }
        __syncthreads();
        int it = 0;
        bool converged = false;
        for (;;) {
            const bool last = it == max_iter || converged;
            // operands of the matrix-core paths from this pass's centers
            if constexpr (BF) center_prep_bf<D>(L, box, k, ldk);
            else if constexpr (MF) center_norms<D>(L, box, k, ldk);
            for (int e = threadIdx.x; e < kd; e += NT) L.s_sum[e] = 0;
            for (int c = threadIdx.x; c < k; c += NT) L.s_cnt[c] = 0;
            if constexpr (BF) {
                // split path: the next piece's raw points load while this one
                // finishes (requested after its products).  On a pass with
                // an update every wavefront takes the block's 64-point pieces
                // from a counter, so that a wavefront that finishes early
                // takes more; the last pass keeps them in place (piece
                // 4 i + wave), since its objective is summed per tile in the
                // fixed order of the plain form.
                const int wave = (int)(threadIdx.x >> 6);
                const uint32_t npc = (uint32_t)(t1 - t0) * 4u;  // pieces of this block
                auto take = [&]() -> uint32_t {
                    uint32_t w = 0;
                    if ((threadIdx.x & 63) == 0) w = atomicAdd(&L.s_next, 1u);
                    return (uint32_t)__builtin_amdgcn_readlane((int)w, 0);
                };
                auto piece_first = [&](uint32_t w) -> int64_t {
                    return (t0 + (int64_t)(w >> 2)) * kAT + (int64_t)(w & 3u) * 64;
                };
                float xr[4][8], xq[4][8];
                unsigned long long nre = 0;
                if (threadIdx.x == 0) {
                    L.s_nu = 0;
                    L.s_next = 4;  // pieces 0..3 go to waves 0..3 below
                }
                uint32_t w = (uint32_t)wave;
                if (w < npc) load_tile_bf<D>(X, piece_first(w), R.n, xr);
                __syncthreads();  // sums, counts, list and counter are set
                while (w < npc) {
                    bf16x8 ah[4], al[4];
                    float xn[4], xa[4][D / 4];
                    const int64_t fw = piece_first(w);
                    split_tile_bf<D>(xr, L.s_mid, fw, R.n, ah, al, xn, xa);
                    const uint32_t wn = last ? w + 4u : take();
                    const int64_t next_w = wn < npc ? piece_first(wn) : -1;
                    const double obj = wave_tile_bf<D>(L, ah, al, xn, xa, xq, next_w, X, fw, R.n, k, ldk,
                                                       lab, !last, shift, nre);
#pragma unroll
                    for (int g = 0; g < 4; ++g)
#pragma unroll
                        for (int e = 0; e < 8; ++e) xr[g][e] = xq[g][e];
                    if (last) {
                        // every wavefront is at piece w of tile w / 4 (in place)
                        const double tot = block_sum_det(obj, L.s_red);
                        if (threadIdx.x == 0) objpart[R.item0 + t0 + (w >> 2)] = tot;
                    }
                    w = wn;
                }
                if (!last) {
                    __syncthreads();  // the list is complete
                    resolve_deferred<D>(L, X, k, ldk, box, lab, shift);
                }
                if ((threadIdx.x & 63) == 0 && nre) atomicAdd(&rs->rechecks, nre);
            } else if constexpr (MF) {
                // the next tile's points are loaded while this one computes
                // (for narrow points; wide ones would need too many registers)
                constexpr bool kPrefetch = D <= 32 && NT == kAT;
                constexpr int TB = NT / kAT;
                const int part = (int)threadIdx.x / kAT;
                const int64_t wofs = ((threadIdx.x & (kAT - 1)) >> 6) * 64;
                float xr[4][D / 4];
                unsigned long long nre = 0;
                if (kPrefetch && t0 + part < t1) load_tile<D>(X, (t0 + part) * kAT + wofs, R.n, xr);
                __syncthreads();  // sums and counts are zeroed
                for (int64_t tb = t0; tb < t1; tb += TB) {
                    const int64_t t = tb + part;  // this part's tile (uniform per wavefront)
                    double obj = 0.0;
                    if (t < t1) {
                        if (!kPrefetch) load_tile<D>(X, t * kAT + wofs, R.n, xr);
                        float xb[4][D / 4], xn[4];
                        center_tile<D>(xr, box, t * kAT + wofs, R.n, xb, xn);
                        if (kPrefetch && t + TB < t1) load_tile<D>(X, (t + TB) * kAT + wofs, R.n, xr);
                        obj = wave_tile_mf<D>(L, xb, xn, X, t * kAT + wofs, R.n, k, ldk, box, lab,
                                              !last, shift, nre);
                    }
                    if (last) {
                        // objective per tile, summed over tiles in order by the
                        // finalize kernel: the same rounding as the plain form
                        const double tot = block_sum_det<NT>(obj, L.s_red);
                        if ((threadIdx.x & (kAT - 1)) == 0 && t < t1) objpart[R.item0 + t] = tot;
                    }
                }
                if ((threadIdx.x & 63) == 0 && nre) atomicAdd(&rs->rechecks, nre);
            } else {
                for (int64_t t = t0; t < t1; ++t) {
                    const double obj = fused_tile<D, MF>(L, X, t * kAT, R.n, d, k, ldk, box, lab,
                                                         !last, shift, &rs->rechecks);
                    if (last) {
                        const double tot = block_sum_det(obj, L.s_red);
                        if (threadIdx.x == 0) objpart[R.item0 + t] = tot;
                    }
                }
            }
            if (last) {
                if (threadIdx.x == 0 && tk.g == 0) rs->iters = it;
                break;
            }
            __syncthreads();
            if (G > 1 && R.xatom) {
                // Shared totals: every block adds its sums into the move's
                // totals with agent-scope integer atomics (performed at the
                // device's coherence point; exact, so any order gives the same
                // bits), waits for them to complete, arrives once, and reads
                // the totals back with agent-scope loads.  Totals rotate over
                // three buffers by move: during move it each block also clears
                // its slice of the buffer of move it + 1, last read as the
                // totals of move it - 2 by blocks that have all since arrived
                // at move it - 1 (this block passed that arrival), and written
                // again only after this move's arrival, which follows the
                // clearing.  The buffer of move 0 is cleared before the launch.
                const int ne = kd + k;
                long long *tb = parts + R.part_off;
                long long *acc = tb + (int64_t)(it % 3) * ne;
                long long *nxt = tb + (int64_t)((it + 1) % 3) * ne;
                for (int e = threadIdx.x; e < kd; e += NT) {
                    const long long v = L.s_sum[e];
                    if (v != 0) __hip_atomic_fetch_add(&acc[e], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                for (int c = threadIdx.x; c < k; c += NT) {
                    const long long v = (long long)L.s_cnt[c];
                    if (v != 0) __hip_atomic_fetch_add(&acc[kd + c], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                {
                    const int S = (ne + G - 1) / G;
                    const int e0 = min(ne, tk.g * S), e1 = min(ne, e0 + S);
                    for (int e = e0 + (int)threadIdx.x; e < e1; e += NT)
                        __hip_atomic_exchange(&nxt[e], 0ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (threadIdx.x == 0) {
                    const uint32_t target = (uint32_t)G * (uint32_t)(it + 1);
                    __hip_atomic_fetch_add(&rs->arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    long long spins = 0;
                    while (__hip_atomic_load(&rs->arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                        __builtin_amdgcn_s_sleep(1);
                        if (++spins > kSpinLimit) {
                            atomicOr(err, 1);
                            break;
                        }
                    }
                }
                __syncthreads();
                for (int e0 = 0; e0 < ne; e0 += NT * kExB) {
                    long long v[kExB];
#pragma unroll
                    for (int u = 0; u < kExB; ++u)
                        v[u] = __hip_atomic_load(&acc[min(e0 + u * NT + (int)threadIdx.x, ne - 1)],
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                    for (int u = 0; u < kExB; ++u) {
                        const int e = e0 + u * NT + (int)threadIdx.x;
                        if (e < kd) L.s_sum[e] = v[u];
                        else if (e < ne) L.s_cnt[e - kd] = (unsigned int)v[u];
                    }
                }
                __syncthreads();
            } else if (G > 1) {
                // Publish this block's sums, wait for the run's other blocks,
                // then sum the parts (exact integer sums: any order gives the
                // same bits), reduce-scattered as below.  The parts and
                // their sums are written and read with agent-scope atomic stores
                // and loads, which the hardware performs at the device's
                // coherence point; every thread waits for its own stores to
                // complete before the block arrives, so a block that sees
                // all arrivals also sees all parts.  No cache-wide fence.
                const int ne = kd + k;
                long long *slot = parts + R.part_off + ((int64_t)(it & 1) * G + tk.g) * ne;
                for (int e = threadIdx.x; e < kd; e += NT)
                    __hip_atomic_store(&slot[e], L.s_sum[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (int c = threadIdx.x; c < k; c += NT)
                    __hip_atomic_store(&slot[kd + c], (long long)L.s_cnt[c], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                // arrive and wait until the run's G blocks have arrived `target` times in all
                auto arrive_wait = [&](uint32_t target) {
                    if (threadIdx.x == 0) {
                        __hip_atomic_fetch_add(&rs->arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        long long spins = 0;
                        while (__hip_atomic_load(&rs->arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                            __builtin_amdgcn_s_sleep(1);
                            if (++spins > kSpinLimit) {
                                atomicOr(err, 1);
                                break;
                            }
                        }
                    }
                    __syncthreads();
                };
                const long long *base = parts + R.part_off + (int64_t)(it & 1) * G * ne;
                // Reduce-scatter: block g sums slice g of the G parts
                // and publishes it; after a second arrival every block
                // reads the summed vector (2 ne words per block instead
                // of G ne).  Parts and sums alternate by iteration
                // parity like the parts alone: a buffer is written again
                // two iterations later, after every block has passed the
                // first arrival of the iteration in between.
                arrive_wait((uint32_t)G * (uint32_t)(2 * it + 1));
                long long *tot = parts + R.part_off + 2ll * G * ne + (int64_t)(it & 1) * ne;
                const int S = (ne + G - 1) / G;
                const int e0 = min(ne, tk.g * S), ns = min(ne, e0 + S) - e0;
                if (G <= 8) {
                    // few parts: every thread sums its elements of the slice
                    // over the G parts in registers, kSumEl elements a round
                    // (loads clamped to valid words, values masked)
                    constexpr int kSumEl = 8;
                    for (int i0 = 0; i0 < ns; i0 += NT * kSumEl) {
                        if (i0 + (int)threadIdx.x >= ns) break;  // no element of this thread
                        long long acc[kSumEl];
#pragma unroll
                        for (int u = 0; u < kSumEl; ++u) acc[u] = 0;
                        for (int q0 = 0; q0 < G; q0 += 2) {
                            long long v[2][kSumEl];
#pragma unroll
                            for (int pq = 0; pq < 2; ++pq)
#pragma unroll
                                for (int u = 0; u < kSumEl; ++u) {
                                    const int q = min(q0 + pq, G - 1);
                                    const int e = min(i0 + u * NT + (int)threadIdx.x, ns - 1);
                                    v[pq][u] = __hip_atomic_load(&base[(int64_t)q * ne + e0 + e], __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
                                }
#pragma unroll
                            for (int pq = 0; pq < 2; ++pq)
#pragma unroll
                                for (int u = 0; u < kSumEl; ++u) acc[u] += q0 + pq < G ? v[pq][u] : 0ll;
                        }
#pragma unroll
                        for (int u = 0; u < kSumEl; ++u) {
                            const int e = i0 + u * NT + (int)threadIdx.x;
                            if (e < ns) __hip_atomic_store(&tot[e0 + e], acc[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
                } else {
                    // many parts (short slices): (element, part) pairs
                    // element-fastest over all threads, kExB loads in flight
                    // each, summed by LDS atomics
                    for (int i = threadIdx.x; i < ns; i += NT) L.s_sum[i] = 0;
                    __syncthreads();
                    const int np = ns * G;
                    for (int p0 = 0; p0 < np; p0 += NT * kExB) {
                        long long v[kExB];
#pragma unroll
                        for (int u = 0; u < kExB; ++u) {
                            const int p = min(p0 + u * NT + (int)threadIdx.x, np - 1);
                            const int q = p / ns, e = p - q * ns;
                            v[u] = __hip_atomic_load(&base[(int64_t)q * ne + e0 + e], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                        }
#pragma unroll
                        for (int u = 0; u < kExB; ++u) {
                            const int p = p0 + u * NT + (int)threadIdx.x;
                            if (p < np) atomicAdd((unsigned long long *)&L.s_sum[p % ns], (unsigned long long)v[u]);
                        }
                    }
                    __syncthreads();
                    for (int i = threadIdx.x; i < ns; i += NT)
                        __hip_atomic_store(&tot[e0 + i], L.s_sum[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                arrive_wait((uint32_t)G * (uint32_t)(2 * it + 2));
                // kExB loads in flight per thread (one at a time, each would
                // wait out the full latency of the coherence point)
                for (int e0 = 0; e0 < ne; e0 += NT * kExB) {
                    long long v[kExB];
#pragma unroll
                    for (int u = 0; u < kExB; ++u)
                        v[u] = __hip_atomic_load(&tot[min(e0 + u * NT + (int)threadIdx.x, ne - 1)],
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                    for (int u = 0; u < kExB; ++u) {
                        const int e = e0 + u * NT + (int)threadIdx.x;
                        if (e < kd) L.s_sum[e] = v[u];
                        else if (e < ne) L.s_cnt[e - kd] = (unsigned int)v[u];
                    }
                }
                __syncthreads();
            }
            const double shift_max = centers_from_sums<D, MF>(L, d, k, ldk, shift, tk.g == 0 ? Cr : nullptr);
            ++it;
            converged = shift_max < tol;
        }
    }
}

// ---------------------------------------------------------------------------
// Plain form, fused path: assign + accumulate over a run's tiles (one item
// per tile), sums flushed to the run's global accumulators with integer
// atomics.
template <int D, bool MF>
__global__ __launch_bounds__(kAT) void k_assign_acc(const float *__restrict__ P,
                                                    const DevRun *__restrict__ runs,
                                                    const Item *__restrict__ items, int item_base,
                                                    const float *__restrict__ C, int32_t *labels,
                                                    RunState *rstate, double *objpart,
                                                    long long *gsum, const uint32_t *__restrict__ boxes,
                                                    int accumulate) {
    __shared__ FusedLds L;
    const Item itm = items[item_base + blockIdx.x];
    const DevRun R = runs[itm.run];
    RunState *rs = rstate + itm.run;
    const int32_t ph = rs->phase;
    if (ph == PH_DONE) return;
    const bool acc = accumulate && ph == PH_ITER;
    const int d = D > 0 ? D : R.d;
    const int k = R.k, kd = k * d, ldk = k + 16;
    const int shift = fix_shift_of(rs->absmax_bits);
    const uint32_t *box = boxes + R.box_off;
    load_centers<MF>(L, C + R.c_off, d, k, ldk);
    for (int e = threadIdx.x; e < kd; e += kAT) L.s_sum[e] = 0;
    for (int c = threadIdx.x; c < k; c += kAT) L.s_cnt[c] = 0;
    __syncthreads();
    if constexpr (MF) center_norms<D>(L, box, k, ldk);
    double obj;
    if constexpr (MF) {
        const int64_t first_w = itm.first + (threadIdx.x >> 6) * 64;
        float xr[4][D / 4], xb[4][D / 4], xn[4];
        unsigned long long nre = 0;
        load_tile<D>(P + R.x_off, first_w, R.n, xr);
        center_tile<D>(xr, box, first_w, R.n, xb, xn);
        obj = wave_tile_mf<D>(L, xb, xn, P + R.x_off, first_w, R.n, k, ldk, box, labels + R.lab_off,
                              acc, shift, nre);
        if ((threadIdx.x & 63) == 0 && nre) atomicAdd(&rs->rechecks, nre);
    } else {
        obj = fused_tile<D, MF>(L, P + R.x_off, itm.first, R.n, d, k, ldk, box, labels + R.lab_off,
                                acc, shift, &rs->rechecks);
    }
    const double tot = block_sum_det(obj, L.s_red);
    if (threadIdx.x == 0) objpart[item_base + blockIdx.x] = tot;
    if (!acc) return;
    long long *gs = gsum + R.sum_off;
    for (int c = threadIdx.x; c < k; c += kAT)
        if (L.s_cnt[c]) atomicAdd((unsigned long long *)&gs[kd + c], (unsigned long long)L.s_cnt[c]);
    for (int e = threadIdx.x; e < kd; e += kAT) {
        const int c = e / d;
        if (L.s_cnt[c])
            atomicAdd((unsigned long long *)&gs[e], (unsigned long long)L.s_sum[sum_idx<D, MF>(c, e - c * d, d)]);
    }
}

// Fused path, per iteration: new centers of run run0 + blockIdx.x from its
// global sums, which the block zeroes for the next iteration.
__global__ __launch_bounds__(kAT) void k_update_fin(const DevRun *__restrict__ runs, int run0,
                                                    float *C, RunState *rstate, long long *gsum,
                                                    double tol) {
    __shared__ FusedLds L;
    const int r = run0 + blockIdx.x;
    const DevRun R = runs[r];
    RunState *rs = rstate + r;
    const int32_t ph = rs->phase;
    if (ph == PH_DONE) return;
    if (ph == PH_FINAL) {
        // the assignment that just ran was the last one of this run
        if (threadIdx.x == 0) rs->phase = PH_DONE;
        return;
    }
    const int d = R.d, k = R.k, kd = k * d;
    const int shift = fix_shift_of(rs->absmax_bits);
    long long *gs = gsum + R.sum_off;
    for (int e = threadIdx.x; e < kd; e += kAT) {
        L.sC[e] = C[R.c_off + e];
        L.s_sum[e] = gs[e];
        gs[e] = 0;
    }
    for (int c = threadIdx.x; c < k; c += kAT) {
        L.s_cnt[c] = (unsigned int)gs[kd + c];
        gs[kd + c] = 0;
    }
    __syncthreads();
    const double mx = centers_from_sums<0, false>(L, d, k, 0, shift, C + R.c_off);
    if (threadIdx.x == 0) {
        rs->iters += 1;
        rs->phase = mx < tol ? PH_FINAL : PH_ITER;
    }
}

// ---------------------------------------------------------------------------
// Scan-update path (k*d beyond the LDS budget): assign without accumulation,
// centers staged through LDS in chunks, rechecks against global memory.
template <int D>
__global__ __launch_bounds__(kAT) void k_assign(const float *__restrict__ P,
                                                const DevRun *__restrict__ runs,
                                                const Item *__restrict__ items, int item_base,
                                                const float *__restrict__ C, int32_t *labels,
                                                RunState *rstate, double *objpart, int last_pass) {
    __shared__ float sC[kLdsFloats];
    __shared__ int32_t s_list[kAT];
    __shared__ int32_t s_newlab[kAT];
    __shared__ uint32_t s_nlist;
    __shared__ double s_red[kAT];
    const Item itm = items[item_base + blockIdx.x];
    const DevRun R = runs[itm.run];
    const int32_t ph = rstate[itm.run].phase;
    if (ph == PH_DONE) return;
    const bool want_obj = last_pass || ph == PH_FINAL;
    const int d = D > 0 ? D : R.d;
    const int k = R.k;
    const int64_t i = itm.first + threadIdx.x;
    const bool valid = i < R.n;
    const float *X = P + R.x_off;
    const float *xg = X + (valid ? i : 0) * d;
    const float *Cr = C + R.c_off;
    float x[D > 0 ? D : 1];
    if (D > 0) {
#pragma unroll
        for (int j = 0; j < D; ++j) x[j] = xg[j];
    }
    if (threadIdx.x == 0) s_nlist = 0;
    float b1 = INFINITY, b2 = INFINITY;
    int32_t i1 = 0;
    const int kc = kLdsFloats / d > 0 ? kLdsFloats / d : 1;
    for (int c0 = 0; c0 < k; c0 += kc) {
        const int nc = kc < k - c0 ? kc : k - c0;
        __syncthreads();
        for (int e = threadIdx.x; e < nc * d; e += kAT) sC[e] = Cr[(int64_t)c0 * d + e];
        __syncthreads();
        scan_centers<D>(x, xg, sC, c0, nc, d, b1, b2, i1);
    }
    const bool certain = certain_gap(b1, b2, d, k);
    if (valid && !certain) s_list[atomicAdd(&s_nlist, 1u)] = threadIdx.x;
    __syncthreads();
    const uint32_t nl = s_nlist;
    recheck_tile(X, itm.first, Cr, d, k, s_list, nl, s_newlab);
    __syncthreads();
    if (valid && !certain) i1 = s_newlab[threadIdx.x];
    double obj = 0.0;
    if (valid) {
        labels[R.lab_off + i] = i1;
        if (want_obj) obj = dist64(xg, Cr + (int64_t)i1 * d, d);
    }
    // an update follows: count the points for their centers
    if (threadIdx.x == 0 && nl) atomicAdd(&rstate[itm.run].rechecks, (unsigned long long)nl);
    if (want_obj) {
        const double tot = block_sum_det(obj, s_red);
        if (threadIdx.x == 0) objpart[item_base + blockIdx.x] = tot;
    }
}

// Chunked path, assignment on matrix cores: the run's centers stream through
// LDS in chunks (dim-major, padded pitch); every wavefront keeps the two
// smallest values of its 64 points across the chunks.  Same centering and
// error bound as stage1_mfma, with max_c ||c - m|| accumulated chunk by
// chunk; near-ties are re-assigned in binary64 against the centers in global
// memory.  The objective of the tile goes to objpart.
template <int D>
__global__ __launch_bounds__(kAT) void k_assign_big(const float *__restrict__ P,
                                                    const DevRun *__restrict__ runs,
                                                    const Item *__restrict__ items, int item_base,
                                                    const float *__restrict__ C, int32_t *labels,
                                                    RunState *rstate, double *objpart,
                                                    const uint32_t *__restrict__ boxes,
                                                    int last_pass) {
    constexpr int KQ = D / 4;
    constexpr int ldc = (kChunkF / D) < 1040 ? (kChunkF / D) : 1040;  // pitch of a staged chunk
    constexpr int kc = ((ldc - 16) / 16) * 16;                         // centers per chunk
    static_assert(kc >= 16, "chunk too small");
    __shared__ float sC[D * ldc];
    __shared__ float cn[ldc];
    __shared__ int32_t s_lab[kAT];
    __shared__ double s_red[kAT];
    const Item itm = items[item_base + blockIdx.x];
    const DevRun R = runs[itm.run];
    RunState *rs = rstate + itm.run;
    const int32_t ph = rs->phase;
    if (ph == PH_DONE) return;
    const bool want_obj = last_pass || ph == PH_FINAL;
    const int k = R.k;
    const float *X = P + R.x_off;
    const float *Cr = C + R.c_off;
    const uint32_t *box = boxes + R.box_off;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kk = lane >> 4;
    const int64_t first_w = itm.first + wave * 64;
    float mq[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) mq[q] = box_mid(box, D, kk + 4 * q);
    float xr[4][KQ];
    load_tile<D>(X, first_w, R.n, xr);
    float xb[4][KQ], xn[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const bool ok = first_w + g * 16 + col < R.n;
        float s2 = 0.0f;
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            const float v = ok ? xr[g][q] - mq[q] : 0.0f;
            xb[g][q] = v;
            s2 = __builtin_fmaf(v, v, s2);
        }
        s2 += lane_xor16(s2);
        s2 += lane_xor32(s2);
        xn[g] = sqrtf(s2);
    }
    float b1[4], b2[4];
    int32_t i1[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        b1[g] = INFINITY;
        b2[g] = INFINITY;
        i1[g] = 0;
    }
    float Rc2 = 0.0f;  // max_c ||c - m||^2 over the chunks seen
    for (int c0 = 0; c0 < k; c0 += kc) {
        const int nc = kc < k - c0 ? kc : k - c0;
        __syncthreads();
        for (int e = threadIdx.x; e < nc * D; e += kAT) {
            const int c = e / D, j = e - c * D;
            sC[j * ldc + c] = Cr[(int64_t)(c0 + c) * D + j];
        }
        __syncthreads();
        float mx = 0.0f;
        for (int c = threadIdx.x; c < ((nc + 15) & ~15); c += kAT) {
            float a = INFINITY;
            if (c < nc) {
                a = 0.0f;
#pragma unroll 4
                for (int j = 0; j < D; ++j) {
                    const float t = sC[j * ldc + c] - box_mid(box, D, j);
                    a = __builtin_fmaf(t, t, a);
                }
                mx = fmaxf(mx, a);
            }
            cn[c] = a;
        }
        s_red[threadIdx.x] = (double)mx;
        __syncthreads();
        for (int st = kAT / 2; st > 0; st >>= 1) {
            if (threadIdx.x < st) s_red[threadIdx.x] = fmax(s_red[threadIdx.x], s_red[threadIdx.x + st]);
            __syncthreads();
        }
        Rc2 = fmaxf(Rc2, (float)s_red[0]);
        for (int t0 = 0; t0 < nc; t0 += 16) {
            const int cA = t0 + col;
            const uint32_t vmask = cA < nc ? 0xFFFFFFFFu : 0u;
            float ca[KQ];
#pragma unroll
            for (int q = 0; q < KQ; ++q) {
                const float cv = sC[(kk + 4 * q) * ldc + cA];
                ca[q] = __uint_as_float(__float_as_uint(-2.0f * (cv - mq[q])) & vmask);
            }
            // the bias of the lane's four output rows starts the accumulator
            const floatx4 cinit = {cn[t0 + 4 * kk], cn[t0 + 4 * kk + 1], cn[t0 + 4 * kk + 2],
                                   cn[t0 + 4 * kk + 3]};
            int32_t ci[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) ci[r] = c0 + t0 + 4 * kk + r;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                floatx4 acc = cinit;
#pragma unroll
                for (int q = 0; q < KQ; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[q], xb[g][q], acc, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float v = acc[r];
                    b2[g] = __builtin_amdgcn_fmed3f(v, b1[g], b2[g]);
                    const bool lt = v < b1[g];
                    b1[g] = lt ? v : b1[g];
                    i1[g] = lt ? ci[r] : i1[g];
                }
            }
        }
    }
    const float Rc = sqrtf(Rc2);
    const float Ku = 2.0f * (float)(D + 5) * 5.9604645e-8f;
    int32_t *wlab = s_lab + wave * 64;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
        for (int o = 16; o <= 32; o <<= 1) {
            const float ob1 = o == 16 ? lane_xor16(b1[g]) : lane_xor32(b1[g]);
            const float ob2 = o == 16 ? lane_xor16(b2[g]) : lane_xor32(b2[g]);
            const int32_t oi = o == 16 ? lane_xor16(i1[g]) : lane_xor32(i1[g]);
            const float nb2 = fminf(fminf(b2[g], ob2), fmaxf(b1[g], ob1));
            const bool take = (ob1 < b1[g]) | ((ob1 == b1[g]) & (oi < i1[g]));  // no branch
            b1[g] = take ? ob1 : b1[g];
            i1[g] = take ? oi : i1[g];
            b2[g] = nb2;
        }
        const float sx = xn[g] + Rc;
        const float E = Ku * sx * sx + 1e-30f;
        const bool certain = k == 1 || (b2[g] - b1[g]) > 2.0f * E;
        if (kk == 0) wlab[g * 16 + col] = i1[g] | (certain ? 0 : (int32_t)0x80000000);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t i = first_w + lane;
    const bool valid = i < R.n;
    const float *xg = X + (valid ? i : 0) * D;
    const int32_t sl = wlab[lane];
    int32_t lab = sl & 0x7fffffff;
    unsigned long long todo = __ballot(valid && sl < 0);
    const unsigned long long nre = (unsigned long long)__popcll(todo);
    while (todo) {
        const int t = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const int32_t w = wave_argmin64(X + (first_w + t) * D, Cr, D, k);
        if (lane == t) lab = w;
    }
    double obj = 0.0;
    if (valid) {
        labels[R.lab_off + i] = lab;
        if (want_obj) obj = dist64(xg, Cr + (int64_t)lab * D, D);
    }
    if (lane == 0 && nre) atomicAdd(&rs->rechecks, nre);
    if (want_obj) {
        const double tot = block_sum_det(obj, s_red);
        if (threadIdx.x == 0) objpart[item_base + blockIdx.x] = tot;
    }
}

// Chunked path on split bfloat16 (D = 8 or 16, rows 16-byte aligned): the
// run's centers stream through LDS in chunks of kBigBfC, each block splitting
// -2 (c - m) into bfloat16 parts as it stages them; stage 1 is the split
// product of stage1_bf (four terms of D attributes in one K = 32 step per
// 8 attributes, accumulator started at ||c - m||^2) with the float32 top-2
// tracking of k_assign_big.  Without the offset Q every partial sum stays
// below 1.03 s^2, s = ||x - m|| + max_c ||c - m||, so the bound of stage1_bf
// holds with Q = 0: E = 2^-16 s^2 + (D + 3 + 2.06 (4 D + 1)) u s^2.  Points
// whose two smallest values are not 2 E apart are re-assigned in binary64
// against the centers in global memory.
constexpr int kBigBfC = 512;  // centers per staged chunk

template <int D>
__global__ __launch_bounds__(kAT) void k_assign_big_bf(const float *__restrict__ P,
                                                       const DevRun *__restrict__ runs,
                                                       const Item *__restrict__ items, int item_base,
                                                       const float *__restrict__ C, int32_t *labels,
                                                       RunState *rstate, double *objpart,
                                                       const uint32_t *__restrict__ boxes,
                                                       int last_pass) {
    static_assert(D == 8 || D == 16, "split chunked path: D = 8 or 16");
    constexpr int S = D / 8;                 // instructions per group and center tile
    constexpr int NA = D >= 16 ? D / 16 : 1;  // distinct A operands per lane
    __shared__ bf16x8 sA[kBigBfC * (D / 4)];
    __shared__ float cn[kBigBfC];
    __shared__ float s_mid[D];
    __shared__ int32_t s_lab[kAT];
    __shared__ double s_red[kAT];
    const Item itm = items[item_base + blockIdx.x];
    const DevRun R = runs[itm.run];
    RunState *rs = rstate + itm.run;
    const int32_t ph = rs->phase;
    if (ph == PH_DONE) return;
    const bool want_obj = last_pass || ph == PH_FINAL;
    const int k = R.k;
    const float *X = P + R.x_off;
    const float *Cr = C + R.c_off;
    const uint32_t *box = boxes + R.box_off;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kg = lane >> 4;
    const int64_t first_w = itm.first + wave * 64;
    if (threadIdx.x < D) s_mid[threadIdx.x] = box_mid(box, D, threadIdx.x);
    __syncthreads();
    float xr[4][8];
    load_tile_bf<D>(X, first_w, R.n, xr);
    bf16x8 ah[4], al[4];
    float xn[4], xa[4][D / 4];
    split_tile_bf<D>(xr, s_mid, first_w, R.n, ah, al, xn, xa);
    int qa[NA];
#pragma unroll
    for (int s = 0; s < NA; ++s) {
        const int t = (32 * s + 8 * kg) / D, j0 = (32 * s + 8 * kg) % D;
        qa[s] = (t & 1) * (D / 8) + j0 / 8;
    }
    bf16x8 b8[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) b8[g] = (D == 8 && kg >= 2) ? al[g] : ah[g];
    float b1[4], b2[4];
    int32_t i1[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        b1[g] = INFINITY;
        b2[g] = INFINITY;
        i1[g] = 0;
    }
    float mx = 0.0f;  // this thread's largest ||c - m||^2 over the centers it staged
    for (int c0 = 0; c0 < k; c0 += kBigBfC) {
        const int nc = kBigBfC < k - c0 ? kBigBfC : k - c0;
        const int ncr = (nc + 15) & ~15;
        __syncthreads();  // nobody still reads the previous chunk
        for (int c = threadIdx.x; c < ncr; c += kAT) {
            float a = INFINITY;
            if (c < nc) {
                a = 0.0f;
                const float *cr = Cr + (int64_t)(c0 + c) * D;
#pragma unroll
                for (int q = 0; q < D / 8; ++q) {
                    bf16x8 hi, lo;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int j = 8 * q + e;
                        const float t = cr[j] - s_mid[j];
                        a = __builtin_fmaf(t, t, a);
                        const float v = -2.0f * t;
                        const __bf16 h = (__bf16)v;
                        hi[e] = h;
                        lo[e] = (__bf16)(v - (float)h);
                    }
                    sA[sa_idx<D>(c, q)] = hi;
                    sA[sa_idx<D>(c, D / 8 + q)] = lo;
                }
                mx = fmaxf(mx, a);
            } else {
                const bf16x8 z = {};
#pragma unroll
                for (int q = 0; q < D / 4; ++q) sA[sa_idx<D>(c, q)] = z;
            }
            cn[c] = a;  // +inf past the run's centers: never selected
        }
        __syncthreads();
        for (int t0 = 0; t0 < ncr; t0 += 16) {
            bf16x8 A[NA];
#pragma unroll
            for (int s = 0; s < NA; ++s) A[s] = sA[sa_idx<D>(t0 + col, qa[s])];
            const floatx4 cinit = {cn[t0 + 4 * kg], cn[t0 + 4 * kg + 1], cn[t0 + 4 * kg + 2],
                                   cn[t0 + 4 * kg + 3]};
            floatx4 acc[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                acc[g] = cinit;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const bf16x8 B = D == 8 ? b8[g] : ((32 * s) / D >= 2 ? al[g] : ah[g]);
                    acc[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[s % NA], B, acc[g], 0, 0, 0);
                }
            }
            const int32_t cb = c0 + t0 + 4 * kg;
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float v = acc[g][r];
                    b2[g] = __builtin_amdgcn_fmed3f(v, b1[g], b2[g]);
                    const bool lt = v < b1[g];
                    b1[g] = lt ? v : b1[g];
                    i1[g] = lt ? cb + r : i1[g];
                }
        }
    }
    const double rmax = block_max<kAT>((double)mx, s_red);
    const float Rc = sqrtf((float)rmax);
    constexpr float Ks = 1.52587890625e-05f;
    constexpr float Ka = (float)(D + 3 + 2.06 * (4 * D + 1)) * 5.9604645e-8f;
    int32_t *wlab = s_lab + wave * 64;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
        for (int o = 16; o <= 32; o <<= 1) {
            const float ob1 = o == 16 ? lane_xor16(b1[g]) : lane_xor32(b1[g]);
            const float ob2 = o == 16 ? lane_xor16(b2[g]) : lane_xor32(b2[g]);
            const int32_t oi = o == 16 ? lane_xor16(i1[g]) : lane_xor32(i1[g]);
            const float nb2 = fminf(fminf(b2[g], ob2), fmaxf(b1[g], ob1));
            const bool take = (ob1 < b1[g]) | ((ob1 == b1[g]) & (oi < i1[g]));  // no branch
            b1[g] = take ? ob1 : b1[g];
            i1[g] = take ? oi : i1[g];
            b2[g] = nb2;
        }
        const float sx = xn[g] + Rc;
        const float s2 = sx * sx;
        const float E = (Ks + Ka) * s2 + 1e-30f;
        const bool certain = k == 1 || (b2[g] - b1[g]) > 2.0f * E;
        if (kg == 0) wlab[g * 16 + col] = i1[g] | (certain ? 0 : (int32_t)0x80000000);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t i = first_w + lane;
    const bool valid = i < R.n;
    const float *xg = X + (valid ? i : 0) * D;
    const int32_t sl = wlab[lane];
    int32_t lab = sl & 0x7fffffff;
    unsigned long long todo = __ballot(valid && sl < 0);
    const unsigned long long nre = (unsigned long long)__popcll(todo);
    while (todo) {
        const int t = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const int32_t w = wave_argmin64(X + (first_w + t) * D, Cr, D, k);
        if (lane == t) lab = w;
    }
    double obj = 0.0;
    if (valid) {
        labels[R.lab_off + i] = lab;
        if (want_obj) obj = dist64(xg, Cr + (int64_t)lab * D, D);
    }
    if (lane == 0 && nre) atomicAdd(&rs->rechecks, nre);
    if (want_obj) {
        const double tot = block_sum_det(obj, s_red);
        if (threadIdx.x == 0) objpart[item_base + blockIdx.x] = tot;
    }
}

// ---------------------------------------------------------------------------
__global__ void k_state_init(RunState *rstate, int R) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    RunState z{};
    z.phase = PH_ITER;
    rstate[r] = z;
}

// Attribute-wise minimum and maximum of every run as ordered bits (box[j],
// box[d + j]) and the largest |x| of the run (grid: chunks x runs).
__global__ void k_box_init(const DevRun *__restrict__ runs, uint32_t *boxes, long long *parts) {
    const DevRun R = runs[blockIdx.x];
    for (int j = threadIdx.x; j < 2 * R.d; j += blockDim.x)
        boxes[R.box_off + j] = j < R.d ? 0xFFFFFFFFu : 0u;
    // batched form with shared totals: the totals of the first move start at zero
    if (R.xatom)
        for (int64_t j = threadIdx.x; j < (int64_t)R.k * R.d + R.k; j += blockDim.x) parts[R.part_off + j] = 0;
}

__global__ __launch_bounds__(256) void k_runbox(const float *__restrict__ P,
                                                const DevRun *__restrict__ runs, uint32_t *boxes,
                                                RunState *rstate) {
    extern __shared__ uint32_t s_box[];  // 2 d words
    __shared__ float s_m[256];
    const DevRun R = runs[blockIdx.y];
    const int d = R.d;
    for (int j = threadIdx.x; j < d; j += 256) {
        s_box[j] = 0xFFFFFFFFu;
        s_box[d + j] = 0u;
    }
    __syncthreads();
    const float *X = P + R.x_off;
    const int64_t per = (R.n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(R.n, r0 + per);
    if (256 % d == 0) {
        // every thread keeps one attribute
        const int col = threadIdx.x % d, rstep = 256 / d;
        uint32_t lo = 0xFFFFFFFFu, hi = 0u;
        for (int64_t row = r0 + threadIdx.x / d; row < r1; row += rstep) {
            const uint32_t o = ordered_bits(X[row * d + col]);
            lo = min(lo, o);
            hi = max(hi, o);
        }
        atomicMin(&s_box[col], lo);
        atomicMax(&s_box[d + col], hi);
    } else {
        for (int64_t row = r0; row < r1; ++row)
            for (int col = threadIdx.x; col < d; col += 256) {
                const uint32_t o = ordered_bits(X[row * d + col]);
                atomicMin(&s_box[col], o);
                atomicMax(&s_box[d + col], o);
            }
    }
    __syncthreads();
    uint32_t *gb = boxes + R.box_off;
    float m = 0.0f;
    for (int j = threadIdx.x; j < d; j += 256) {
        if (s_box[j] != 0xFFFFFFFFu) {
            atomicMin(&gb[j], s_box[j]);
            atomicMax(&gb[d + j], s_box[d + j]);
            m = fmaxf(m, fmaxf(fabsf(ordered_float(s_box[j])), fabsf(ordered_float(s_box[d + j]))));
        }
    }
    s_m[threadIdx.x] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) s_m[threadIdx.x] = fmaxf(s_m[threadIdx.x], s_m[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && s_m[0] > 0.0f)
        atomicMax(&rstate[blockIdx.y].absmax_bits, __float_as_uint(s_m[0]));
}

__global__ void k_fill_i64(long long *a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
}

// first k points of every run as its starting centers (mode 1), or the
// strided start C[q] = X[q * floor(n / k)] (mode 2)
__global__ void k_init(const float *__restrict__ P, const DevRun *__restrict__ runs, float *C,
                       int mode) {
    const DevRun R = runs[blockIdx.y];
    const int64_t tot = (int64_t)R.k * R.d;
    const int64_t stride = mode == 2 ? R.n / R.k : 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = e / R.d, j = e - q * R.d;
        C[R.c_off + e] = P[R.x_off + q * stride * R.d + j];
    }
}

// Objective of every run: the per-tile partials summed in a fixed order (each
// thread a contiguous range, then a fixed tree), one block per run.
__global__ __launch_bounds__(kAT) void k_finalize(const DevRun *__restrict__ runs,
                                                  const RunState *__restrict__ rstate,
                                                  const double *__restrict__ objpart,
                                                  int32_t *iters, double *sse,
                                                  unsigned long long *rechecks) {
    __shared__ double s_red[kAT];
    const int r = blockIdx.x;
    const DevRun D = runs[r];
    const int per = (D.nitems + kAT - 1) / kAT;
    const int q0 = threadIdx.x * per, q1 = min(D.nitems, q0 + per);
    double s = 0.0;
    for (int q = q0; q < q1; ++q) s = s + objpart[D.item0 + q];
    const double tot = block_sum_det(s, s_red);
    if (threadIdx.x == 0) {
        sse[D.orig] = tot;
        if (iters) iters[D.orig] = rstate[r].iters;
        if (rechecks) atomicAdd(rechecks, rstate[r].rechecks);
    }
}

// ---------------------------------------------------------------------------
#define SUBKM_DISPATCH_D(d, FN, ...)                                                      \
    switch (d) {                                                                          \
        case 1: return FN<1>(__VA_ARGS__);                                                \
        case 2: return FN<2>(__VA_ARGS__);                                                \
        case 4: return FN<4>(__VA_ARGS__);                                                \
        case 8: return FN<8>(__VA_ARGS__);                                                \
        case 16: return FN<16>(__VA_ARGS__);                                              \
        case 32: return FN<32>(__VA_ARGS__);                                              \
        case 64: return FN<64>(__VA_ARGS__);                                              \
        case 128: return FN<128>(__VA_ARGS__);                                            \
        default: return FN<0>(__VA_ARGS__);                                               \
    }

// matrix-core variants exist for attribute counts that are multiples of 4
template <int D>
constexpr bool kHasMF = D >= 4 && D <= 128 && D % 4 == 0;

template <int D>
subkm_status launch_assign_acc(subkm_ctx *ctx, bool mf, int nitems, int item_base, const float *P,
                               const DevRun *runs, const Item *items, const float *C,
                               int32_t *labels, RunState *rs, double *objpart, long long *gsum,
                               const uint32_t *boxes, int accumulate) {
    ProfScope ps(ctx, PK_ASSIGN);
    if constexpr (kHasMF<D>) {
        if (mf) {
            hipLaunchKernelGGL((k_assign_acc<D, true>), dim3(nitems), dim3(kAT), 0, ctx->stream, P,
                               runs, items, item_base, C, labels, rs, objpart, gsum, boxes, accumulate);
            SUBKM_LAUNCHED(ctx);
            return SUBKM_OK;
        }
    }
    hipLaunchKernelGGL((k_assign_acc<D, false>), dim3(nitems), dim3(kAT), 0, ctx->stream, P, runs,
                       items, item_base, C, labels, rs, objpart, gsum, boxes, accumulate);
    SUBKM_LAUNCHED(ctx);
    return SUBKM_OK;
}

template <int D>
subkm_status launch_assign(subkm_ctx *ctx, int nitems, int item_base, const float *P,
                           const DevRun *runs, const Item *items, const float *C, int32_t *labels,
                           RunState *rs, double *objpart, int last_pass) {
    ProfScope ps(ctx, PK_ASSIGN);
    hipLaunchKernelGGL(k_assign<D>, dim3(nitems), dim3(kAT), 0, ctx->stream, P, runs, items,
                       item_base, C, labels, rs, objpart, last_pass);
    SUBKM_LAUNCHED(ctx);
    return SUBKM_OK;
}

// Threads per block of the persistent kernel (every path: 256; the kernel
// also takes 512-thread blocks, two 256-point tiles at a time, which gave no
// gain where registers allowed four wavefronts per SIMD).
template <int D, bool MF, bool BF>
constexpr int persist_nt() {
    return kAT;
}

// mf: 0 vector path, 1 float32 matrix cores, 2 split bfloat16 matrix cores
template <int D, bool MF, bool BF>
subkm_status launch_persist_k(subkm_ctx *ctx, int blocks, const float *P, const DevRun *runs,
                              const Task *tasks, const int32_t *task_off, float *C,
                              int32_t *labels, RunState *rs, long long *parts, double *objpart,
                              const uint32_t *boxes, int max_iter, double tol, int *err) {
    ProfScope ps(ctx, PK_LLOYD_FUSED);
    void *args[] = {(void *)&P,       (void *)&runs,   (void *)&tasks, (void *)&task_off,
                    (void *)&C,       (void *)&labels, (void *)&rs,    (void *)&parts,
                    (void *)&objpart, (void *)&boxes,  (void *)&max_iter, (void *)&tol,
                    (void *)&err};
    constexpr int NT = persist_nt<D, MF, BF>();
    SUBKM_HIP(ctx, hipLaunchCooperativeKernel((const void *)k_lloyd_persist<D, MF, BF, NT>, dim3(blocks),
                                              dim3(NT), args, 0, ctx->stream));
    return SUBKM_OK;
}

template <int D>
subkm_status launch_persist(subkm_ctx *ctx, int mf, int blocks, const float *P,
                            const DevRun *runs, const Task *tasks, const int32_t *task_off,
                            float *C, int32_t *labels, RunState *rs, long long *parts,
                            double *objpart, const uint32_t *boxes, int max_iter, double tol,
                            int *err) {
    if constexpr (kBF<D>) {
        if (mf == 2)
            return launch_persist_k<D, true, true>(ctx, blocks, P, runs, tasks, task_off, C, labels, rs,
                                                   parts, objpart, boxes, max_iter, tol, err);
    }
    if constexpr (kHasMF<D>) {
        if (mf)
            return launch_persist_k<D, true, false>(ctx, blocks, P, runs, tasks, task_off, C, labels, rs,
                                                    parts, objpart, boxes, max_iter, tol, err);
    }
    return launch_persist_k<D, false, false>(ctx, blocks, P, runs, tasks, task_off, C, labels, rs, parts,
                                             objpart, boxes, max_iter, tol, err);
}

template <int D, bool MF, bool BF>
int persist_occupancy_k() {
    constexpr int NT = persist_nt<D, MF, BF>();
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_lloyd_persist<D, MF, BF, NT>, NT, 0) !=
        hipSuccess) {
        hipGetLastError();
        return 0;
    }
    return nb;
}

template <int D>
int persist_occupancy(int mf) {
    if constexpr (kBF<D>) {
        if (mf == 2) return persist_occupancy_k<D, true, true>();
    }
    if constexpr (kHasMF<D>) {
        if (mf) return persist_occupancy_k<D, true, false>();
    }
    return persist_occupancy_k<D, false, false>();
}

int persist_occupancy_d(int d, int mf) { SUBKM_DISPATCH_D(d, persist_occupancy, mf); }

template <int D>
int persist_tiles_per_step(int mf) {
    if constexpr (kHasMF<D>) {
        if (mf == 1) return persist_nt<D, true, false>() / kAT;
    }
    return 1;
}

// 256-point tiles a persistent block of this path takes at a time
int persist_tiles_per_step_d(int d, int mf) { SUBKM_DISPATCH_D(d, persist_tiles_per_step, mf); }

subkm_status assign_acc_d(subkm_ctx *ctx, int d, bool mf, int nitems, int item_base,
                          const float *P, const DevRun *runs, const Item *items, const float *C,
                          int32_t *labels, RunState *rs, double *objpart, long long *gsum,
                          const uint32_t *boxes, int accumulate) {
    if (nitems <= 0) return SUBKM_OK;
    SUBKM_DISPATCH_D(d, launch_assign_acc, ctx, mf, nitems, item_base, P, runs, items, C, labels,
                     rs, objpart, gsum, boxes, accumulate);
}

template <int D>
subkm_status launch_assign_big(subkm_ctx *ctx, int nitems, int item_base, const float *P,
                               const DevRun *runs, const Item *items, const float *C,
                               int32_t *labels, RunState *rs, double *objpart,
                               const uint32_t *boxes, int last_pass, int bf) {
    if constexpr (D == 8 || D == 16) {
        if (bf) {
            ProfScope ps(ctx, PK_ASSIGN);
            hipLaunchKernelGGL(k_assign_big_bf<D>, dim3(nitems), dim3(kAT), 0, ctx->stream, P, runs,
                               items, item_base, C, labels, rs, objpart, boxes, last_pass);
            SUBKM_LAUNCHED(ctx);
            return SUBKM_OK;
        }
    }
    if constexpr (kHasMF<D>) {
        ProfScope ps(ctx, PK_ASSIGN);
        hipLaunchKernelGGL(k_assign_big<D>, dim3(nitems), dim3(kAT), 0, ctx->stream, P, runs, items,
                           item_base, C, labels, rs, objpart, boxes, last_pass);
        SUBKM_LAUNCHED(ctx);
        return SUBKM_OK;
    } else {
        return launch_assign<D>(ctx, nitems, item_base, P, runs, items, C, labels, rs, objpart,
                                last_pass);
    }
}

// assignment of runs beyond the LDS budget: matrix cores when d allows
subkm_status assign_big_d(subkm_ctx *ctx, int d, int nitems, int item_base, const float *P,
                          const DevRun *runs, const Item *items, const float *C, int32_t *labels,
                          RunState *rs, double *objpart, const uint32_t *boxes, int last_pass,
                          int bf) {
    if (nitems <= 0) return SUBKM_OK;
    SUBKM_DISPATCH_D(d, launch_assign_big, ctx, nitems, item_base, P, runs, items, C, labels, rs,
                     objpart, boxes, last_pass, bf);
}

subkm_status persist_d(subkm_ctx *ctx, int d, int mf, int blocks, const float *P,
                       const DevRun *runs, const Task *tasks, const int32_t *task_off, float *C,
                       int32_t *labels, RunState *rs, long long *parts, double *objpart,
                       const uint32_t *boxes, int max_iter, double tol, int *err) {
    SUBKM_DISPATCH_D(d, launch_persist, ctx, mf, blocks, P, runs, tasks, task_off, C, labels, rs,
                     parts, objpart, boxes, max_iter, tol, err);
}

// Largest-work-first schedule of the runs of one attribute count over
// `blocks` persistent blocks.  Run r gets G_r blocks (about its share of the
// total work, at most one per tile) and starts when its G_r least-loaded
// blocks are free.  Every block's task list follows the global assignment
// order, so the per-run barriers cannot wait on each other in a cycle.
void schedule(const std::vector<int> &rr, const std::vector<DevRun> &dr, int blocks,
              bool exchange, int gcap, int tpb, int step, std::vector<int32_t> &G,
              std::vector<std::vector<Task>> &per_block) {
    std::vector<int> order(rr);
    auto work = [&](int r) { return (double)dr[r].n * dr[r].k * dr[r].d; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
    double total = 0;
    for (int r : order) total += work(r);
    const double target = total / blocks;
    using Slot = std::pair<double, int>;  // (finish time, block)
    std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> pq;
    for (int b = 0; b < blocks; ++b) pq.push({0.0, b});
    per_block.assign(blocks, {});
    for (int r : order) {
        const int64_t tiles = (dr[r].n + kAT - 1) / kAT;
        int64_t g = std::llround(work(r) / std::max(target, 1.0));
        // with a per-iteration exchange every move ends in two barriers of
        // the run's G blocks: keep G at most gcap and at least tpb tiles per
        // block; never fewer tiles per block than a block takes at a time
        const int64_t per = std::max(std::max(1, tpb), step);
        const int64_t gmax =
            exchange ? std::min<int64_t>(std::min(gcap, kMaxG), std::max<int64_t>(1, tiles / per))
                     : (tiles + step - 1) / step;
        g = std::max<int64_t>(1, std::min<int64_t>({g, gmax, (int64_t)blocks}));
        G[r] = (int32_t)g;
        std::vector<Slot> take;
        double start = 0;
        for (int64_t q = 0; q < g; ++q) {
            take.push_back(pq.top());
            pq.pop();
            start = std::max(start, take.back().first);
        }
        const double fin = start + work(r) / g;
        for (int64_t q = 0; q < g; ++q) {
            per_block[take[q].second].push_back(Task{r, (int32_t)q});
            pq.push({fin, take[q].second});
        }
    }
}

}  // namespace

// Per-run path and the per-run parts of the scratch layout of one call
// (shared by the call and by the bound of its scratch).
struct PlanSizes {
    bool all_fused = true;
    int64_t sum_words = 0, box_words = 0, cnt_words = 0, order_words = 0, frag_words = 0, cn_words = 0;
};

void plan_runs(const subkm_run *runs, int32_t R, int32_t precision, int32_t max_iter,
               std::vector<DevRun> &dr, PlanSizes &z) {
    dr.assign(R, DevRun{});
    for (int r = 0; r < R; ++r) {
        const subkm_run &u = runs[r];
        DevRun &D = dr[r];
        std::memset(&D, 0, sizeof D);
        D.x_off = u.x_off;
        D.n = u.n;
        D.c_off = u.c_off;
        D.lab_off = u.lab_off;
        D.d = u.d;
        D.k = u.k;
        const int64_t kd = (int64_t)u.k * u.d;
        const bool mf_shape = (u.d == 4 || u.d == 8 || u.d == 16 || u.d == 32 || u.d == 64 || u.d == 128);
        D.mf = (mf_shape && (int64_t)u.d * (u.k + 16) <= kCF) ? 1 : 0;
        // split bfloat16 matrix cores where D allows (16-byte row loads: the
        // caller's pointer alignment is checked per call, see lloyd_run)
        if (D.mf && (u.d == 8 || u.d == 16 || u.d == 32)) D.mf = 2;
        D.fused = (kd <= kSumW && kd <= kCF && u.k <= kMaxK) ? 1 : 0;
        // a run with moves whose tiles would overload the kMaxG blocks that
        // can share one run's partial sums takes the wide path, whose update
        // scales with the number of points
        if (max_iter > 0 && u.n > kHugeRun) D.fused = 0;
        z.all_fused = z.all_fused && D.fused;
        D.box_off = z.box_words;
        z.box_words += 2 * (int64_t)u.d;
        if (D.fused) {
            D.sum_off = z.sum_words;
            z.sum_words += kd + u.k;
        } else {
            if (u.d <= kWalkD) {
                // sums of the centers that cross a walk window
                D.sum_off = z.sum_words;
                z.sum_words += kd;
            }
            // centers stream from memory; exact update through labels
            D.cnt_off = z.cnt_words;
            z.cnt_words += 3 * (int64_t)u.k;
            z.order_words = std::max<int64_t>(z.order_words, u.lab_off + u.n);
            // split bfloat16 for 32 attributes under either setting (one
            // matrix-core step covers the row; same labels as float32),
            // and for up to 128 attributes under SUBKM_PREC_BF16
            D.split = ((u.d == 32 || (precision == SUBKM_PREC_BF16 && u.d >= 32 && u.d <= 128)) &&
                       u.k <= 1024) ? 1 : 0;
            if (D.split) {
                const int64_t kt = ceil_div(u.k, 16), st = ceil_div(u.d, 32);
                D.frag_off = z.frag_words;
                z.frag_words += kt * st * 128;
                D.cn_off = z.cn_words;
                z.cn_words += kt * 16;
            }
        }
    }
}

// bytes requested per scratch slot by the call's plan
void plan_requests(int32_t R, int64_t n_items, int64_t n_tasks, int64_t n_toff, int64_t n_obj,
                   int64_t part_words, const PlanSizes &z, size_t *req) {
    auto need = [&](int slot, size_t b) { req[slot] = std::max(req[slot], b); };
    need(SC_RUNS, sizeof(DevRun) * R + sizeof(Item) * n_items + sizeof(Task) * n_tasks +
                      sizeof(int32_t) * n_toff + 64);
    need(SC_RSTATE, sizeof(RunState) * R + 64);
    need(SC_SSEPART, sizeof(double) * (n_obj + 1));
    need(SC_FIXSCALE, sizeof(long long) * (z.sum_words + part_words + 1));
    need(SC_RECHECK, 128);
    need(SC_BOX, sizeof(uint32_t) * (z.box_words + 1));
    need(SC_WCNT, sizeof(int32_t) * (z.cnt_words + 2));
    need(SC_WORDER, sizeof(int32_t) * (2 * z.order_words + 1));
    need(SC_FRAGS, sizeof(uint4) * (z.frag_words + 1));
    need(SC_CNORM, sizeof(float) * (z.cn_words + 16));
}

// One call with a given schedule of the batched form (the schedule changes
// no result: sums are exact integers and labels exact).
subkm_status lloyd_run(subkm_ctx *ctx, const float *P, const subkm_run *runs, int32_t R,
                       float *C, int32_t *labels, int32_t max_iter, double tol,
                       int32_t precision, int32_t form, int32_t *iters, double *sse,
                       int init_mode, unsigned long long *rechecks_acc, const LloydSched &sc) {
    hipStream_t s = ctx->stream;
    // runs of one path are launched together: order them by path (outputs go
    // back to the caller's order through DevRun::orig)
    std::vector<int> ord(R);
    for (int r = 0; r < R; ++r) ord[r] = r;
    {
        std::vector<DevRun> probe;
        PlanSizes pz;
        plan_runs(runs, R, precision, max_iter, probe, pz);
        auto key = [&](int r) {
            const DevRun &D = probe[r];
            return std::make_tuple(D.fused, D.split, D.d, D.mf);
        };
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return key(a) < key(b); });
    }
    std::vector<subkm_run> sorted_runs(R);
    for (int r = 0; r < R; ++r) sorted_runs[r] = runs[ord[r]];
    runs = sorted_runs.data();
    std::vector<DevRun> dr;
    PlanSizes z;
    plan_runs(runs, R, precision, max_iter, dr, z);
    for (int r = 0; r < R; ++r) dr[r].orig = ord[r];
    {
        // the split path loads 16-byte row pieces: with any run's rows not
        // 16-byte aligned, every such run takes the float32 matrix cores
        bool aligned = true;
        for (int r = 0; r < R; ++r)
            if (dr[r].mf == 2 && ((uintptr_t)(P + dr[r].x_off) & 15u)) aligned = false;
        if (!aligned)
            for (int r = 0; r < R; ++r)
                if (dr[r].mf == 2) dr[r].mf = 1;
    }
    int64_t sum_words = z.sum_words, box_words = z.box_words, cnt_words = z.cnt_words;
    const int64_t order_words = z.order_words, frag_words = z.frag_words, cn_words = z.cn_words;
    std::vector<std::pair<int, int>> ds;  // distinct (attribute count, matrix-core path)
    for (int r = 0; r < R; ++r) ds.push_back({dr[r].d, dr[r].mf});
    std::sort(ds.begin(), ds.end());
    ds.erase(std::unique(ds.begin(), ds.end()), ds.end());

    // Batched form: the runs whose centers and sums fit on chip go to one
    // persistent launch per (d, matrix-core) group; the others (sorted
    // first) take the per-phase path, in the same call.  Plain form: every
    // run on its own, one launch per phase.
    const bool batched = form == SUBKM_FORM_BATCHED;
    int nwide = 0;
    while (nwide < R && !dr[nwide].fused) ++nwide;
    const bool persist_any = batched && nwide < R;
    const int nplain = batched ? nwide : R;  // runs that take per-phase launches
    std::vector<Item> items;
    std::vector<int> walk0(R, 0), nwalk(R, 0);
    std::vector<Task> tasks;
    std::vector<int32_t> task_off;
    struct Group {
        int d, mf, block0, blocks;
    };
    std::vector<Group> groups;
    int64_t part_words = 0;
    int n_obj = 0;
    // per-phase runs: assignment items (tiles) first, so that an item's index
    // is also its objective slot; then update and walk items of wide runs
    for (int r = 0; r < nplain; ++r) {
        DevRun &D = dr[r];
        D.item0 = (int)items.size();
        for (int64_t f = 0; f < D.n; f += kAT) items.push_back(Item{r, (int32_t)f, 0, 0});
        D.nitems = (int)items.size() - D.item0;
    }
    n_obj = (int)items.size();
    for (int r = 0; r < nplain; ++r) {
        DevRun &D = dr[r];
        D.uitem0 = (int)items.size();
        if (!D.fused) {
            // walked runs whose centers average under a quarter window
            // (few cross a window edge) read 256 centers per block
            D.kcu = (D.d <= kWalkD && D.n < (int64_t)D.k * (kWalkW / 4)) ? kWalkCenters : kWideCenters;
            for (int c = 0; c < D.k; c += D.kcu) items.push_back(Item{r, c, 0, 0});
        }
        D.nuitems = (int)items.size() - D.uitem0;
    }
    // Points per wavefront in the update walk: narrow points share a
    // wavefront (fewer idle lanes), as long as the walk launch keeps about
    // kWalkMinBlocks blocks; the batched form launches the walks of all its
    // wide runs together, the plain form one run at a time.
    {
        int64_t walked = 0;
        for (int r = 0; r < nplain; ++r)
            if (!dr[r].fused && dr[r].d <= kWalkD) walked += dr[r].n;
        for (int r = 0; r < nplain; ++r) {
            DevRun &D = dr[r];
            D.wpp = 1;
            if (D.fused || D.d > kWalkD) continue;
            const int64_t tot = batched ? walked : D.n;
            const int cap = 64 / walk_lanes(D.d);
            while (2 * D.wpp <= cap && tot >= (int64_t)kWalkB * 2 * D.wpp * kWalkMinBlocks) D.wpp *= 2;
        }
    }
    for (int r = 0; r < nplain; ++r) {
        walk0[r] = (int)items.size();
        if (!dr[r].fused && dr[r].d <= kWalkD)
            for (int64_t f = 0; f < dr[r].n; f += (int64_t)kWalkB * dr[r].wpp)
                items.push_back(Item{r, (int32_t)f, 0, 0});
        nwalk[r] = (int)items.size() - walk0[r];
    }
    if (persist_any) {
        // one persistent launch per attribute count, at most the co-resident capacity
        std::vector<std::pair<int, int>> dsf;
        for (int r = nwide; r < R; ++r) dsf.push_back({dr[r].d, dr[r].mf});
        std::sort(dsf.begin(), dsf.end());
        dsf.erase(std::unique(dsf.begin(), dsf.end()), dsf.end());
        int block_base = 0;
        task_off.push_back(0);
        for (auto dm : dsf) {
            const int dv = dm.first, mv = dm.second;
            std::vector<int> rr;
            int64_t tiles = 0;
            for (int r = nwide; r < R; ++r)
                if (dr[r].d == dv && dr[r].mf == mv) {
                    rr.push_back(r);
                    tiles += (dr[r].n + kAT - 1) / kAT;
                }
            const int occ = std::max(1, persist_occupancy_d(dv, mv));
            const int step = persist_tiles_per_step_d(dv, mv);
            const int64_t cap = std::max<int64_t>(1, (int64_t)ctx->cu_count * occ / std::max(1, sc.bdiv));
            const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(cap, (tiles + step - 1) / step));
            std::vector<int32_t> G(R, 1);
            std::vector<std::vector<Task>> pb;
            schedule(rr, dr, blocks, max_iter > 0, sc.gcap, sc.tpb, step, G, pb);
            // shared totals only while the atomics of one move stay few (a
            // single split run: the final run of the mid workload adds 139k
            // words per move and saves a barrier and the slice sums); with
            // millions per move (the 128 local runs: 2.2M) they gained nothing
            // measurable over the published parts, which such calls keep
            int64_t xvol = 0;
            for (int r : rr)
                if (G[r] > 1) xvol += (int64_t)G[r] * ((int64_t)dr[r].k * dr[r].d + dr[r].k);
            const bool xat = sc.xmode == 1 && max_iter > 0 && xvol <= kXAtomMax;
            for (int r : rr) {
                DevRun &D = dr[r];
                D.G = G[r];
                D.nitems = (int32_t)((D.n + kAT - 1) / kAT);
                D.part_off = part_words;
                // exchange slots only when there is an update to exchange:
                // published parts and slice sums, or three rotating totals
                D.xatom = (G[r] > 1 && xat) ? 1 : 0;
                if (G[r] > 1 && max_iter > 0)
                    part_words += (D.xatom ? 3ll : 2ll * G[r] + 2) * ((int64_t)D.k * D.d + D.k);
            }
            for (int b = 0; b < blocks; ++b) {
                for (const Task &t : pb[b]) tasks.push_back(t);
                task_off.push_back((int32_t)tasks.size());
            }
            groups.push_back(Group{dv, mv, block_base, blocks});
            block_base += blocks;
        }
        // objective slots of the persistent runs follow the per-phase items
        for (int r = nwide; r < R; ++r) {
            dr[r].item0 = n_obj;
            n_obj += dr[r].nitems;
        }
    }
    const int n_items = (int)items.size();

    // device copies of the plan: runs | items | tasks | task_off
    const size_t b_runs = sizeof(DevRun) * R, b_items = sizeof(Item) * n_items;
    const size_t b_tasks = sizeof(Task) * tasks.size(), b_toff = sizeof(int32_t) * task_off.size();
    const size_t b_plan = b_runs + b_items + b_tasks + b_toff;
    size_t req[SC_COUNT] = {};
    plan_requests(R, n_items, (int64_t)tasks.size(), (int64_t)task_off.size(), n_obj, part_words, z, req);
    char *d_plan = (char *)ctx_scratch(ctx, SC_RUNS, req[SC_RUNS]);
    RunState *d_rs = (RunState *)ctx_scratch(ctx, SC_RSTATE, req[SC_RSTATE]);
    double *d_obj = (double *)ctx_scratch(ctx, SC_SSEPART, req[SC_SSEPART]);
    long long *d_sum = (long long *)ctx_scratch(ctx, SC_FIXSCALE, req[SC_FIXSCALE]);
    int *d_err = (int *)ctx_scratch(ctx, SC_RECHECK, req[SC_RECHECK]);
    uint32_t *d_box = (uint32_t *)ctx_scratch(ctx, SC_BOX, req[SC_BOX]);
    int32_t *d_cnt = (int32_t *)ctx_scratch(ctx, SC_WCNT, req[SC_WCNT]);
    // point indices grouped by label, then their labels
    int32_t *d_order = (int32_t *)ctx_scratch(ctx, SC_WORDER, req[SC_WORDER]);
    uint4 *d_frags = (uint4 *)ctx_scratch(ctx, SC_FRAGS, req[SC_FRAGS]);
    float *d_cn = (float *)ctx_scratch(ctx, SC_CNORM, req[SC_CNORM]);
    if (!d_plan || !d_rs || !d_obj || !d_sum || !d_err || !d_box || !d_cnt || !d_order || !d_frags || !d_cn)
        return SUBKM_ENOMEM;
    int stage = 0;
    char *h = (char *)ctx_stage(ctx, b_plan + 64, &stage);
    if (!h) return ctx->err.empty() ? SUBKM_ENOMEM : SUBKM_EDEVICE;
    DevRun *d_runs = (DevRun *)d_plan;
    Item *d_items = (Item *)(d_plan + b_runs);
    Task *d_tasks = (Task *)(d_plan + b_runs + b_items);
    int32_t *d_toff = (int32_t *)(d_plan + b_runs + b_items + b_tasks);
    // the plan goes through a slot of the staging ring (no wait for the
    // stream: only the copy issued from the same slot calls ago must be done)
    std::memcpy(h, dr.data(), b_runs);
    if (b_items) std::memcpy(h + b_runs, items.data(), b_items);
    if (b_tasks) std::memcpy(h + b_runs + b_items, tasks.data(), b_tasks);
    if (b_toff) std::memcpy(h + b_runs + b_items + b_tasks, task_off.data(), b_toff);
    SUBKM_HIP(ctx, hipMemcpyAsync(d_plan, h, b_plan, hipMemcpyHostToDevice, s));
    SUBKM_TRY(ctx_stage_issued(ctx, stage));

    hipLaunchKernelGGL(k_state_init, dim3(ceil_div(R, 256)), dim3(256), 0, s, d_rs, R);
    SUBKM_LAUNCHED(ctx);
    hipLaunchKernelGGL(k_fill_i64, dim3(std::min<int64_t>(ceil_div(sum_words + 1, 256), 2048)),
                       dim3(256), 0, s, d_sum, sum_words + 1);
    SUBKM_LAUNCHED(ctx);
    if (cnt_words) {
        const int64_t w = ceil_div(cnt_words, 2);
        hipLaunchKernelGGL(k_fill_i64, dim3(std::min<int64_t>(ceil_div(w, 256), 2048)), dim3(256), 0, s,
                           (long long *)d_cnt, w);
        SUBKM_LAUNCHED(ctx);
    }
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, s, (long long *)d_err, 16);
    SUBKM_LAUNCHED(ctx);
    {
        // attribute-wise bounds of every run: reference point of the
        // matrix-core paths and fixed-point scale of the sums
        int64_t nmax = 0;
        int dmax = 1;
        for (int r = 0; r < R; ++r) {
            nmax = std::max<int64_t>(nmax, dr[r].n);
            dmax = std::max(dmax, dr[r].d);
        }
        hipLaunchKernelGGL(k_box_init, dim3(R), dim3(256), 0, s, d_runs, d_box, d_sum + sum_words);
        SUBKM_LAUNCHED(ctx);
        hipLaunchKernelGGL(k_runbox, dim3(std::min<int64_t>(ceil_div(nmax, 2048), 1024), R), dim3(256),
                           2 * sizeof(uint32_t) * dmax, s, P, d_runs, d_box, d_rs);
        SUBKM_LAUNCHED(ctx);
    }
    if (init_mode) {
        int64_t kmax = 0;
        for (int r = 0; r < R; ++r) kmax = std::max<int64_t>(kmax, (int64_t)runs[r].k * runs[r].d);
        hipLaunchKernelGGL(k_init, dim3(std::min<int64_t>(ceil_div(kmax, 256), 1024), R), dim3(256),
                           0, s, P, d_runs, C, init_mode);
        SUBKM_LAUNCHED(ctx);
    }
    long long *gsum = d_sum;
    long long *parts = d_sum + sum_words;
    unsigned long long *d_rechecks = (unsigned long long *)(d_err + 16);

    // one assignment launch for runs [r0, r1), which share path and attribute count
    auto assign_seg = [&](int r0, int r1, int a) -> subkm_status {
        const DevRun &D0 = dr[r0];
        const int i0 = D0.item0, ni = dr[r1 - 1].item0 + dr[r1 - 1].nitems - i0;
        const int last = a == max_iter ? 1 : 0;
        if (D0.fused)
            return assign_acc_d(ctx, D0.d, D0.mf != 0, ni, i0, P, d_runs, d_items, C, labels, d_rs, d_obj,
                                gsum, d_box, a < max_iter ? 1 : 0);
        if (D0.split) {
            int kt = 0;
            for (int r = r0; r < r1; ++r) kt = std::max(kt, (int)ceil_div(dr[r].k, 16));
            const int S = (int)ceil_div(D0.d, 32);
            SUBKM_TRY(wide_split_prep(ctx, r0, r1 - r0, kt, S, d_runs, C, d_box, d_frags, d_cn, d_rs));
            return wide_assign_split(ctx, S, i0, ni, P, d_runs, d_items, C, d_frags, d_cn, labels, d_rs,
                                     d_obj, d_box, last);
        }
        // 8 or 16 attributes with 16-byte aligned rows: split bfloat16 stage 1
        bool bf = D0.d == 8 || D0.d == 16;
        for (int r = r0; bf && r < r1; ++r)
            if ((uintptr_t)(P + dr[r].x_off) & 15u) bf = false;
        return assign_big_d(ctx, D0.d, ni, i0, P, d_runs, d_items, C, labels, d_rs, d_obj, d_box, last,
                            bf ? 1 : 0);
    };
    // one update for runs [r0, r1), all on-chip or all wide
    auto update_seg = [&](int r0, int r1) -> subkm_status {
        if (dr[r0].fused) {
            ProfScope ps(ctx, PK_UPDATE);
            hipLaunchKernelGGL(k_update_fin, dim3(r1 - r0), dim3(kAT), 0, s, d_runs, r0, C, d_rs, gsum, tol);
            SUBKM_LAUNCHED(ctx);
            return SUBKM_OK;
        }
        const int i0 = dr[r0].item0, ni = dr[r1 - 1].item0 + dr[r1 - 1].nitems - i0;
        const int u0 = dr[r0].uitem0, nu = dr[r1 - 1].uitem0 + dr[r1 - 1].nuitems - u0;
        const int w0 = walk0[r0], nw = walk0[r1 - 1] + nwalk[r1 - 1] - w0;
        return wide_update(ctx, r0, r1 - r0, i0, ni, w0, nw, u0, nu, P, d_runs, d_items, labels, C, d_rs,
                           d_cnt, d_order, order_words, gsum, tol);
    };
    auto same_assign = [&](int a, int b) {
        return dr[a].d == dr[b].d && dr[a].fused == dr[b].fused && dr[a].mf == dr[b].mf &&
               dr[a].split == dr[b].split;
    };

    if (persist_any) {
        std::unique_lock<std::mutex> gate;
        if (ctx->coop) {
            gate = std::unique_lock<std::mutex>(ctx->coop->mu);
            if (ctx->coop->armed) SUBKM_HIP(ctx, hipStreamWaitEvent(s, ctx->coop->ev, 0));
        }
        // a barrier that gives up sets the context's sticky flag, which
        // subkm_synchronize reports
        for (const Group &g : groups)
            SUBKM_TRY(persist_d(ctx, g.d, g.mf, g.blocks, P, d_runs, d_tasks, d_toff + g.block0,
                                C, labels, d_rs, parts, d_obj, d_box, max_iter, tol, ctx->sticky));
        if (ctx->coop) {
            SUBKM_HIP(ctx, hipEventRecord(ctx->coop->ev, s));
            ctx->coop->armed = true;
        }
    }
    if (form == SUBKM_FORM_PLAIN) {
        // one run at a time, one launch per phase
        for (int r = 0; r < R; ++r) {
            for (int a = 0; a <= max_iter; ++a) {
                SUBKM_TRY(assign_seg(r, r + 1, a));
                if (a == max_iter) break;
                SUBKM_TRY(update_seg(r, r + 1));
            }
        }
    } else if (nwide > 0) {
        // the batched form's runs beyond the on-chip budget: every phase is
        // one launch per group of consecutive runs of the same path
        for (int a = 0; a <= max_iter; ++a) {
            for (int r0 = 0; r0 < nwide;) {
                int r1 = r0 + 1;
                while (r1 < nwide && same_assign(r0, r1)) ++r1;
                SUBKM_TRY(assign_seg(r0, r1, a));
                r0 = r1;
            }
            if (a == max_iter) break;
            SUBKM_TRY(update_seg(0, nwide));
        }
    }
    hipLaunchKernelGGL(k_finalize, dim3(R), dim3(kAT), 0, s, d_runs, d_rs, d_obj, iters, sse,
                       rechecks_acc ? rechecks_acc : d_rechecks);
    SUBKM_LAUNCHED(ctx);
    return SUBKM_OK;
}

// ---------------------------------------------------------------------------
// Schedule tuner of the batched form.  A shape is (runs, points, smallest
// and largest d and k, precision, moves or not); on the first call of a new
// shape with tuning on, every candidate schedule runs the call itself on the
// caller's data (restarting from the same centers), the fastest is kept for
// the shape, and the call is made once more with it.  Results are identical
// under every schedule, so tuning only changes the time.
namespace {
// (a few blocks per run suit calls of one or few runs, whose time is the
// per-move exchange among their blocks)
const LloydSched kCandidates[] = {{64, 1, 2, 0}, {32, 1, 2, 0},  {16, 1, 2, 0}, {64, 2, 2, 0},
                                  {32, 2, 2, 0}, {16, 2, 2, 0},  {128, 1, 1, 0}, {64, 1, 1, 0},
                                  {8, 1, 2, 0},  {4, 1, 2, 0},   {128, 1, 1, 1}, {64, 1, 2, 1},
                                  {32, 1, 2, 1}, {16, 1, 2, 1}};

TuneKey shape_key(const subkm_run *runs, int32_t R, int32_t precision, int32_t max_iter) {
    int64_t npts = 0;
    int32_t dmin = INT32_MAX, dmax = 0, kmin = INT32_MAX, kmax = 0;
    for (int r = 0; r < R; ++r) {
        npts += runs[r].n;
        dmin = std::min(dmin, runs[r].d);
        dmax = std::max(dmax, runs[r].d);
        kmin = std::min(kmin, runs[r].k);
        kmax = std::max(kmax, runs[r].k);
    }
    TuneKey k;
    k.v[0] = (uint64_t)R;
    k.v[1] = (uint64_t)npts;
    k.v[2] = ((uint64_t)(uint32_t)dmin << 32) | (uint32_t)dmax;
    k.v[3] = ((uint64_t)(uint32_t)kmin << 32) | (uint32_t)kmax;
    k.v[4] = ((uint64_t)(uint32_t)precision << 1) | (max_iter > 0 ? 1u : 0u);
    return k;
}
}  // namespace

subkm_status lloyd_impl(subkm_ctx *ctx, const float *P, const subkm_run *runs, int32_t R,
                        float *C, int32_t *labels, int32_t max_iter, double tol,
                        int32_t precision, int32_t form, int32_t *iters, double *sse,
                        int init_mode, unsigned long long *rechecks_acc) {
    const LloydSched def = kCandidates[0];
    if (form != SUBKM_FORM_BATCHED || max_iter <= 0 || (!ctx->tune_on && ctx->tune.empty()))
        return lloyd_run(ctx, P, runs, R, C, labels, max_iter, tol, precision, form, iters, sse,
                         init_mode, rechecks_acc, def);
    const TuneKey key = shape_key(runs, R, precision, max_iter);
    auto it = ctx->tune.find(key);
    if (it != ctx->tune.end())
        return lloyd_run(ctx, P, runs, R, C, labels, max_iter, tol, precision, form, iters, sse,
                         init_mode, rechecks_acc, it->second.sched);
    if (!ctx->tune_on)
        return lloyd_run(ctx, P, runs, R, C, labels, max_iter, tol, precision, form, iters, sse,
                         init_mode, rechecks_acc, def);
    hipStream_t s = ctx->stream;
    // the caller's starting centers, restored before every candidate
    size_t cfloats = 0;
    for (int r = 0; r < R; ++r)
        cfloats = std::max<size_t>(cfloats, (size_t)runs[r].c_off + (size_t)runs[r].k * runs[r].d);
    float *saved = nullptr;
    if (init_mode == 0) {
        saved = (float *)ctx_scratch(ctx, SC_TUNE, cfloats * sizeof(float));
        if (!saved) return SUBKM_ENOMEM;
        SUBKM_HIP(ctx, hipMemcpyAsync(saved, C, cfloats * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    TuneEntry best{def, 1e300};
    for (const LloydSched &sc : kCandidates) {
        if (saved)
            SUBKM_HIP(ctx, hipMemcpyAsync(C, saved, cfloats * sizeof(float), hipMemcpyDeviceToDevice, s));
        SUBKM_HIP(ctx, hipEventRecord(ctx->ev[6], s));
        SUBKM_TRY(lloyd_run(ctx, P, runs, R, C, labels, max_iter, tol, precision, form, iters, sse,
                            init_mode, nullptr, sc));
        SUBKM_HIP(ctx, hipEventRecord(ctx->ev[7], s));
        SUBKM_HIP(ctx, hipEventSynchronize(ctx->ev[7]));
        float ms = 0.0f;
        SUBKM_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev[6], ctx->ev[7]));
        if (ms < best.ms) best = TuneEntry{sc, (double)ms};
    }
    ctx->tune[key] = best;
    if (saved) SUBKM_HIP(ctx, hipMemcpyAsync(C, saved, cfloats * sizeof(float), hipMemcpyDeviceToDevice, s));
    return lloyd_run(ctx, P, runs, R, C, labels, max_iter, tol, precision, form, iters, sse, init_mode,
                     rechecks_acc, best.sched);
}

// Upper bound of the scratch one lloyd_impl call requests per slot (for
// admission control): the same per-run plan; the batched schedule, which
// depends on the device, is bounded by its largest possible size.
void lloyd_scratch_requests(const subkm_run *runs, int32_t R, int32_t precision, int32_t form,
                            int32_t max_iter, int cu_count, size_t *req) {
    std::vector<DevRun> dr;
    PlanSizes z;
    plan_runs(runs, R, precision, max_iter, dr, z);
    int64_t tiles = 0, n_items = 0, n_tasks = 0, n_toff = 0, part_words = 0;
    for (int r = 0; r < R; ++r) tiles += ceil_div(dr[r].n, kAT);
    const bool batched = form == SUBKM_FORM_BATCHED;
    // runs of the persistent launch (batched form, on-chip runs): tasks and
    // exchange slots; every other run: per-phase items
    std::vector<std::pair<int, int>> ds;
    for (int r = 0; r < R; ++r) {
        const int64_t t = ceil_div(dr[r].n, kAT);
        if (batched && dr[r].fused) {
            ds.push_back({dr[r].d, dr[r].mf});
            const int64_t g = max_iter > 0 ? std::min<int64_t>(kMaxG, std::max<int64_t>(1, t)) : t;
            n_tasks += g;
            if (max_iter > 0 && g > 1)
                part_words += (2 * g + 2) * ((int64_t)dr[r].k * dr[r].d + dr[r].k);
        } else {
            n_items += t;
            if (!dr[r].fused) {
                n_items += ceil_div(dr[r].k, kWideCenters);  // at most
                if (dr[r].d <= kWalkD) n_items += ceil_div(dr[r].n, kWalkB);  // at most
            }
        }
    }
    std::sort(ds.begin(), ds.end());
    ds.erase(std::unique(ds.begin(), ds.end()), ds.end());
    if (!ds.empty()) {
        n_toff = 1;
        for (auto dm : ds) {
            int64_t gt = 0;
            for (int r = 0; r < R; ++r)
                if (dr[r].fused && dr[r].d == dm.first && dr[r].mf == dm.second) gt += ceil_div(dr[r].n, kAT);
            n_toff += std::max<int64_t>(1, std::min<int64_t>((int64_t)cu_count * 32, gt));
        }
    }
    plan_requests(R, n_items, n_tasks, n_toff, tiles, part_words, z, req);
}
