// Unequal sized subclustering (Sec. III, Algorithm 2).
//
// The m landmarks lie evenly on the segment from the corner point L (the
// attribute-wise minimum of the points, step 2) to H (the attribute-wise
// maximum, step 3), both ends included:
//     p_q[j] = L[j] + (q / (m - 1)) * (H[j] - L[j])      (binary64, in that order)
// and m = 1 gives the single landmark L.  Every point joins the landmark at
// the least binary64 squared distance (attributes left to right, no FMA), the
// lower q on a tie (step 5).  Groups follow landmark order, members ascending
// index; a group may be empty.
//
// Kernels (one HBM pass to find the groups, one to move the rows):
//   minmax_impl     L and H (exact column minima and maxima), unless the
//                   caller knows them from the scaling of S;
//   k_uq_prep       one block: L and H - L in binary64 and float32, and the
//                   bounds used by the certified search below;
//   k_uq_landmarks  the landmarks, only when the caller asks for them;
//   k_uq_assign     one block per segment of consecutive points: the nearest
//                   landmark of every point and the segment's histogram,
//                   stored landmark-major, counts[q * nseg + s];
//   k_uq_scan_blocks exclusive scan of counts in that order, per block of
//                   4096 cells, with the block sums;
//   k_uq_scatter    one block per segment: the scanned block sums (every
//                   block rescans them in LDS) complete the scan, so that
//                   cell (q, s) is the first output position of group q's
//                   members in segment s (segment 0's cells are the group
//                   offsets); then stable placement of perm and of the rows
//                   of P (wave ballots rank equal groups in index order,
//                   waves take turns in index order).
//
// The nearest landmark without visiting all m.  With P(t) = L + t (H - L)
// (exact arithmetic, the binary64 H - L), the squared distance
// g(t) = ||x - P(t)||^2 is a convex quadratic in t.  A float32 projection of
// x on the segment guesses q0; the binary64 distances f(q) of the window
// q0 - 1 .. q0 + 1 are evaluated exactly as the definition does, and the
// window [a, z] is widened one landmark at a time until both sides are
// certified.  With u = 2^-53, the binary64 landmark p_q is within
// eps = u sqrt(sum_j (|L_j| + 2.01 |H_j - L_j|)^2) of P(t_q), and f(q) is
// within a relative (d + 2) u / (1 - (d + 2) u) of ||x - p_q||^2.  From
// these, lo(q) <= sqrt(g(t_q)) <= hi(q) are computed from f(q) alone.  The
// right side is certified when z = m - 1, or when
//     lo(z) > hi(z - 1)                        (g increases from t_z on)
//     (1 - gam) (lo(z) - eps) > sqrt(f(b)) (1 + gam)   (so f(q) > f(b), q > z)
// with b the window's best; the left side is the mirror image.  Every
// landmark outside a certified window has a binary64 distance strictly above
// f(b), so the window's argmin (lower q on ties) is the argmin over all m,
// bit for bit.  The bounds carry a factor 2 and a few ulps of slack for the
// rounding of their own evaluation.
//
// With the Manhattan distance the same search holds with the distance itself
// in place of its square root: ||x - P(t)||_1 is convex in t (a sum of
// convex functions), the landmark rounding moves it by at most
// eps = u sum_j (|L_j| + 2.01 |H_j - L_j|), and the evaluated sum of d
// non-negative rounded terms is within the same relative bound.
#include "internal.h"

#include <algorithm>
#include <cmath>

#pragma clang fp contract(off)

namespace {

constexpr int kUT = 256;                   // threads per block
constexpr int64_t kMaxCounts = 1ll << 22;  // histogram cells (segments x landmarks)
constexpr int kScanPer = 16;               // scan elements per thread
constexpr int kScanBlock = kUT * kScanPer;
constexpr int kScanPartsMax = 1024;        // kMaxCounts / kScanBlock
constexpr double kU = 1.1102230246251565e-16;  // 2^-53

struct UqParam {
    double eps;    // bound of ||p_q - P(t_q)|| (times 2)
    double gam;    // relative bound of the evaluated distances (with slack)
    float inv_n2;  // 1 / sum_j Df_j^2 in float32 (the guess only), 0 if none
    int32_t flat;  // every H_j == L_j: all landmarks are L
};

// Block sum of one value per thread in a fixed order (deterministic).
template <typename T>
__device__ T block_sum_fixed(T v, T *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kUT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + s];
        __syncthreads();
    }
    T r = sh[0];
    __syncthreads();
    return r;
}

// The landmark basis.  With xmin/xmax (the column bounds of the data S was
// min-max scaled from) the corners are known exactly: L_j = 0 and H_j = 1
// (0 for a constant column), since the scaling maps the minimum to 0 and the
// maximum to 1 without rounding.
__global__ __launch_bounds__(kUT) void k_uq_prep(const float *__restrict__ mins,
                                                 const float *__restrict__ maxs,
                                                 const float *__restrict__ xmin,
                                                 const float *__restrict__ xmax, int d,
                                                 double *__restrict__ Ld, double *__restrict__ Dd,
                                                 float *__restrict__ Lf, float *__restrict__ Df,
                                                 int metric, UqParam *prm) {
    __shared__ double shd[kUT];
    __shared__ float shf[kUT];
    __shared__ int shi[kUT];
    double sl = 0.0, sa = 0.0;
    float sf = 0.0f;
    int nz = 0;
    for (int j = threadIdx.x; j < d; j += kUT) {
        const float lo = xmin ? 0.0f : mins[j];
        const float hi = xmin ? (xmax[j] > xmin[j] ? 1.0f : 0.0f) : maxs[j];
        const double l = (double)lo;
        const double dd = (double)hi - (double)lo;
        const float df = (float)dd;
        Ld[j] = l;
        Dd[j] = dd;
        Lf[j] = lo;
        Df[j] = df;
        const double a = fabs(l) + 2.01 * dd;
        sl = sl + a * a;
        sa = sa + a;
        sf = sf + df * df;
        nz |= dd != 0.0;
    }
    const double SL = block_sum_fixed(sl, shd);
    const double SA = block_sum_fixed(sa, shd);
    const float SF = block_sum_fixed(sf, shf);
    const int NZ = block_sum_fixed(nz, shi);
    if (threadIdx.x == 0) {
        UqParam p;
        // squared Euclidean: the bound of ||e||_2; Manhattan: of ||e||_1
        p.eps = 2.0 * kU * (metric ? SA : sqrt(SL)) * (1.0 + 8.0 * kU);
        const double du = (double)(d + 2) * kU;
        p.gam = 2.0 * du / (1.0 - du) + 16.0 * kU;
        p.inv_n2 = SF > 0.0f ? 1.0f / SF : 0.0f;
        p.flat = NZ == 0;
        *prm = p;
    }
}

__global__ __launch_bounds__(kUT) void k_uq_landmarks(const double *__restrict__ Ld,
                                                      const double *__restrict__ Dd, int d,
                                                      int64_t m, double *__restrict__ out) {
    const int64_t total = m * d;
    for (int64_t e = (int64_t)blockIdx.x * kUT + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kUT) {
        const int64_t q = e / d;
        const int j = (int)(e - q * d);
        const double t = m == 1 ? 0.0 : (double)q / (double)(m - 1);
        out[e] = Ld[j] + t * Dd[j];
    }
}

// A point's row as the search reads it.  each(f) calls f(value, j) for the
// attributes in ascending j (the order every sum below needs).
//   RowReg<R>: d = 4 * n4 floats, n4 <= R, loaded into registers at once
//              (all loads in flight together, both passes from registers);
//   RowVec:    d = 4 * n4 floats read from memory in float4 units;
//   RowScalar: any d, read float by float.
template <int R>
struct RowReg {
    float4 v[R];
    int n4;
    __host__ __device__ __forceinline__ RowReg(const float *x, int d) : n4(d >> 2) {
        const float4 *x4 = (const float4 *)x;
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (k < n4) v[k] = x4[k];
    }
    template <class F>
    __host__ __device__ __forceinline__ void each(F &&f) const {
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (k < n4) {
                f(v[k].x, 4 * k);
                f(v[k].y, 4 * k + 1);
                f(v[k].z, 4 * k + 2);
                f(v[k].w, 4 * k + 3);
            }
    }
};

struct RowVec {
    const float4 *x4;
    int n4;
    __host__ __device__ __forceinline__ RowVec(const float *x, int d)
        : x4((const float4 *)x), n4(d >> 2) {}
    template <class F>
    __host__ __device__ __forceinline__ void each(F &&f) const {
#pragma unroll 4
        for (int k = 0; k < n4; ++k) {
            const float4 v = x4[k];
            f(v.x, 4 * k);
            f(v.y, 4 * k + 1);
            f(v.z, 4 * k + 2);
            f(v.w, 4 * k + 3);
        }
    }
};

struct RowScalar {
    const float *x;
    int d;
    __host__ __device__ __forceinline__ RowScalar(const float *p, int dd) : x(p), d(dd) {}
    template <class F>
    __host__ __device__ __forceinline__ void each(F &&f) const {
#pragma unroll 4
        for (int j = 0; j < d; ++j) f(x[j], j);
    }
};

// binary64 distance of the row to the landmark at t: M = 0 squared
// Euclidean, M = 1 Manhattan (attributes left to right; the landmark
// coordinate is formed exactly as in its definition).
template <int M>
__host__ __device__ __forceinline__ double uq_term(double q) {
    return M ? fabs(q) : q * q;
}

template <int M, class Row>
__host__ __device__ __forceinline__ double uq_dist(const Row &x, const double *__restrict__ Ld,
                                                   const double *__restrict__ Dd, double t) {
    double acc = 0.0;
    x.each([&](float xv, int j) {
        const double q = (double)xv - (Ld[j] + t * Dd[j]);
        acc = acc + uq_term<M>(q);
    });
    return acc;
}

// The same for three landmarks in one pass over the row.
template <int M, class Row>
__host__ __device__ __forceinline__ void uq_dist3(const Row &x, const double *__restrict__ Ld,
                                                  const double *__restrict__ Dd, double t0,
                                                  double t1, double t2, double &f0, double &f1,
                                                  double &f2) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    x.each([&](float xv, int j) {
        const double xd = (double)xv, l = Ld[j], dj = Dd[j];
        double q;
        q = xd - (l + t0 * dj);
        a0 = a0 + uq_term<M>(q);
        q = xd - (l + t1 * dj);
        a1 = a1 + uq_term<M>(q);
        q = xd - (l + t2 * dj);
        a2 = a2 + uq_term<M>(q);
    });
    f0 = a0;
    f1 = a1;
    f2 = a2;
}

// Nearest landmark of the row (the lower q on ties), by the certified window
// search described at the top of this file (host-callable, so that the
// search can be exercised on the CPU).  x serves the guess and the first
// window; xm, the same row, the rare widening steps (a memory-backed row, so
// that no register copy of the row stays live through the loop).
template <int M, class Row, class RowM>
__host__ __device__ int uq_nearest(const Row &x, const RowM &xm, int m,
                                   const double *__restrict__ Ld,
                                   const double *__restrict__ Dd, const float *__restrict__ Lf,
                                   const float *__restrict__ Df, const UqParam &P) {
    if (m == 1 || P.flat) return 0;  // every landmark is the same point
    const int m1 = m - 1;
    const double dm1 = (double)m1;
    // the guess: float32 projection of x on the segment
    float dot = 0.0f;
    x.each([&](float xv, int j) { dot = fmaf(xv - Lf[j], Df[j], dot); });
    const float u = dot * P.inv_n2 * (float)m1;
    int q0 = 0;
    if (u > 0.0f) q0 = u < (float)m1 ? (int)rintf(u) : m1;  // NaN gives 0
    int a = q0 > 0 ? q0 - 1 : 0;
    int z = q0 < m1 ? q0 + 1 : m1;
    double fa, fa1, fz1, fz, fb;
    int b;
    {
        double f0, f1, f2;
        const double t0 = (double)a / dm1, t1 = (double)(a + 1) / dm1, t2 = (double)z / dm1;
        uq_dist3<M>(x, Ld, Dd, t0, t1, t2, f0, f1, f2);
        // window of three (a, a+1, z) or of two (a, z = a+1, f2 == f1)
        fa = f0;
        fa1 = f1;
        fz = f2;
        fz1 = z - a == 2 ? f1 : f0;
        b = a;
        fb = f0;
        if (f1 < fb) {
            fb = f1;
            b = a + 1;
        }
        if (f2 < fb) {
            fb = f2;
            b = z;
        }
    }
    const double cl = 1.0 - P.gam, ch = 1.0 + P.gam;
    const double dn = 1.0 - 4.0 * kU, up = 1.0 + 4.0 * kU;
    const double eps = P.eps;
    // bounds of the exact distance to the ideal landmark: of its square root
    // for the squared Euclidean distance, of itself for the Manhattan one
    auto root = [](double f) { return M ? f : sqrt(f); };
    auto lo = [&](double f) { return fmax(0.0, (root(f) * cl - eps) * dn); };
    auto hi = [&](double f) { return (root(f) * ch + eps) * up; };
    for (;;) {
        const double rb = root(fb) * ch * up;
        if (z < m1) {
            const double lz = lo(fz);
            if (!(lz > hi(fz1) && (lz - eps) * cl * dn > rb)) {
                ++z;
                fz1 = fz;
                fz = uq_dist<M>(xm, Ld, Dd, (double)z / dm1);
                if (fz < fb) {
                    fb = fz;
                    b = z;
                }
                continue;
            }
        }
        if (a > 0) {
            const double la = lo(fa);
            if (!(la > hi(fa1) && (la - eps) * cl * dn > rb)) {
                --a;
                fa1 = fa;
                fa = uq_dist<M>(xm, Ld, Dd, (double)a / dm1);
                if (fa <= fb) {
                    fb = fa;
                    b = a;
                }
                continue;
            }
        }
        break;
    }
    return b;
}

// Row kinds of the assignment kernel: registers for d = 4 n4 up to 4 R, else
// float4 or scalar reads.
template <int K>
struct RowOf;
template <>
struct RowOf<0> {
    using T = RowScalar;
};
template <>
struct RowOf<1> {
    using T = RowVec;
};
template <>
struct RowOf<8> {
    using T = RowReg<8>;
};
template <>
struct RowOf<16> {
    using T = RowReg<16>;
};
template <>
struct RowOf<32> {
    using T = RowReg<32>;
};

template <int K, int M>
__global__ __launch_bounds__(kUT) void k_uq_assign(const float *__restrict__ S, int64_t n, int d,
                                                   int m, int64_t seg, int64_t nseg,
                                                   const double *__restrict__ Ld,
                                                   const double *__restrict__ Dd,
                                                   const float *__restrict__ Lf,
                                                   const float *__restrict__ Df,
                                                   const UqParam *__restrict__ prm,
                                                   int32_t *__restrict__ group,
                                                   uint32_t *__restrict__ counts) {
    using Row = typename RowOf<K>::T;
    extern __shared__ uint32_t h[];  // m
    const UqParam P = *prm;
    for (int q = threadIdx.x; q < m; q += kUT) h[q] = 0;
    __syncthreads();
    const int64_t s = blockIdx.x;
    const int64_t i0 = s * seg, i1 = i0 + seg < n ? i0 + seg : n;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kUT) {
        const Row x(S + i * d, d);
        int q;
        if (K == 0)
            q = uq_nearest<M>(x, x, m, Ld, Dd, Lf, Df, P);
        else
            q = uq_nearest<M>(x, RowVec(S + i * d, d), m, Ld, Dd, Lf, Df, P);
        group[i] = q;
        atomicAdd(&h[q], 1u);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < m; q += kUT) counts[(int64_t)q * nseg + s] = h[q];
}

// Exclusive scan of one value per thread across the block; *total gets the sum.
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
        if (k < w) before += sh[k];
        all += sh[k];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

__global__ __launch_bounds__(kUT) void k_uq_scan_blocks(uint32_t *__restrict__ v, int64_t E,
                                                        uint32_t *__restrict__ part) {
    __shared__ uint32_t sh[kUT / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
    uint32_t loc[kScanPer];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const uint32_t x = base + k < E ? v[base + k] : 0u;
        loc[k] = sum;
        sum += x;
    }
    uint32_t total;
    const uint32_t ex = block_excl_scan(sum, sh, &total);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < E) v[base + k] = ex + loc[k];
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

template <int V>
struct VecOf;
template <>
struct VecOf<1> {
    using T = float;
};
template <>
struct VecOf<4> {
    using T = float4;
};

template <int V>
__global__ __launch_bounds__(kUT) void k_uq_scatter(const float *__restrict__ S, int64_t n, int d,
                                                    int m, int nbits, int64_t seg, int64_t nseg,
                                                    const int32_t *__restrict__ group,
                                                    const uint32_t *__restrict__ pos0,
                                                    const uint32_t *__restrict__ part, int np,
                                                    float *__restrict__ P,
                                                    int32_t *__restrict__ perm,
                                                    int64_t *__restrict__ offsets) {
    using VT = typename VecOf<V>::T;
    extern __shared__ uint32_t next[];  // m: next output position of each group
    __shared__ uint32_t s_part[kScanPartsMax];
    __shared__ uint32_t s_pos[kUT];
    __shared__ uint32_t s_tmp[kUT / 64];
    const int64_t s = blockIdx.x;
    // exclusive scan of the scan blocks' sums (small: every block redoes it)
    {
        constexpr int per = kScanPartsMax / kUT;
        uint32_t v[per], sum = 0;
#pragma unroll
        for (int k = 0; k < per; ++k) {
            const int e = threadIdx.x * per + k;
            v[k] = e < np ? part[e] : 0u;
            sum += v[k];
        }
        uint32_t total;
        uint32_t run = block_excl_scan(sum, s_tmp, &total);
#pragma unroll
        for (int k = 0; k < per; ++k) {
            s_part[threadIdx.x * per + k] = run;
            run += v[k];
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < m; q += kUT) {
        const int64_t e = (int64_t)q * nseg + s;
        next[q] = pos0[e] + s_part[e / kScanBlock];
        if (s == 0) offsets[q] = next[q];  // group q starts in segment 0
    }
    if (s == 0 && threadIdx.x == 0) offsets[m] = n;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t i0 = s * seg, i1 = i0 + seg < n ? i0 + seg : n;
    const int dv = d / V;
    // row copy: rows of up to kUT vectors are spread rpp rows per pass
    const int rpp = dv <= kUT ? kUT / dv : 0;
    const int cr = dv <= kUT ? threadIdx.x / dv : 0;
    const int cc = dv <= kUT ? threadIdx.x - cr * dv : 0;
    for (int64_t c0 = i0; c0 < i1; c0 += kUT) {
        const int64_t i = c0 + threadIdx.x;
        const bool valid = i < i1;
        const int q = valid ? group[i] : 0;
        // lanes of this wave with the same group
        unsigned long long same = __ballot(valid);
        for (int bit = 0; bit < nbits; ++bit) {
            const bool on = (q >> bit) & 1;
            const unsigned long long bb = __ballot(on);
            same &= on ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(same & below);
        const uint32_t cnt = (uint32_t)__popcll(same);
        uint32_t pos = 0;
        for (int t = 0; t < kUT / 64; ++t) {  // waves in index order
            if (w == t && valid) {
                pos = next[q] + rank;
                if (rank == 0) next[q] = pos + cnt;
            }
            __syncthreads();
        }
        if (valid) {
            perm[pos] = (int32_t)i;
            s_pos[threadIdx.x] = pos;
        }
        __syncthreads();
        const int nrow = (int)(i1 - c0 < kUT ? i1 - c0 : kUT);
        const VT *src = (const VT *)(S + c0 * d);
        VT *dst = (VT *)P;
        if (rpp > 0) {
            if (cr < rpp)
                for (int r = cr; r < nrow; r += rpp)
                    dst[(int64_t)s_pos[r] * dv + cc] = src[(int64_t)r * dv + cc];
        } else {
            for (int r = 0; r < nrow; ++r)
                for (int c = threadIdx.x; c < dv; c += kUT)
                    dst[(int64_t)s_pos[r] * dv + c] = src[(int64_t)r * dv + c];
        }
        __syncthreads();
    }
}

struct UqBufs {
    float *mins, *maxs, *Lf, *Df;
    double *Ld, *Dd;
    UqParam *prm;
    uint32_t *part, *counts;
    int *flag;
    int32_t *group;
};

struct UqPlan {
    int64_t seg, nseg, E;
    int np;
};

UqPlan uq_plan(int64_t n, int64_t m) {
    UqPlan p;
    // about 2048 segments or more (8 blocks per CU), up to 16 points per thread
    int64_t ppt = 1;
    while (ppt < 16 && ceil_div(n, (int64_t)kUT * ppt * 2) >= 2048) ppt *= 2;
    p.seg = kUT * ppt;
    while (m * ceil_div(n, p.seg) > kMaxCounts) p.seg *= 2;
    p.nseg = ceil_div(n, p.seg);
    p.E = m * p.nseg;
    p.np = (int)ceil_div(p.E, kScanBlock);
    return p;
}

size_t uq_bytes(int64_t n, int32_t d, int64_t m, size_t *group_bytes) {
    const UqPlan p = uq_plan(n, m);
    *group_bytes = (size_t)n * sizeof(int32_t);
    return 256 + (size_t)d * (4 * sizeof(float) + 2 * sizeof(double)) + sizeof(UqParam) +
           (size_t)(p.np + 1) * sizeof(uint32_t) + (size_t)p.E * sizeof(uint32_t) + 4 * 64;
}

}  // namespace

void unequal_scratch_requests(int64_t n, int32_t d, int64_t m, size_t *req) {
    size_t gb = 0;
    const size_t cb = uq_bytes(n, d, m, &gb);
    req[SC_UQ] = std::max(req[SC_UQ], cb);
    req[SC_UQ_GROUP] = std::max(req[SC_UQ_GROUP], gb);
    req[SC_MM_PART] = std::max(req[SC_MM_PART], minmax_scratch_bytes(n, d));
}

subkm_status subcluster_unequal_impl(subkm_ctx *ctx, const float *S, int64_t n, int32_t d,
                                     int64_t m, float *P, int32_t *perm, int64_t *offsets,
                                     double *landmarks, int32_t metric, const float *xmin,
                                     const float *xmax) {
    ProfScope ps(ctx, PK_SUBCLUSTER);
    const UqPlan pl = uq_plan(n, m);
    size_t gbytes = 0;
    const size_t cbytes = uq_bytes(n, d, m, &gbytes);
    char *c = (char *)ctx_scratch(ctx, SC_UQ, cbytes);
    int32_t *group = (int32_t *)ctx_scratch(ctx, SC_UQ_GROUP, gbytes);
    if (!c || !group) return SUBKM_ENOMEM;
    // carve (every piece 64-byte aligned)
    auto take = [&](size_t bytes) {
        char *p = c;
        c += (bytes + 63) & ~(size_t)63;
        return (void *)p;
    };
    UqBufs b;
    b.flag = (int *)take(256);
    b.mins = (float *)take((size_t)d * 4);
    b.maxs = (float *)take((size_t)d * 4);
    b.Lf = (float *)take((size_t)d * 4);
    b.Df = (float *)take((size_t)d * 4);
    b.Ld = (double *)take((size_t)d * 8);
    b.Dd = (double *)take((size_t)d * 8);
    b.prm = (UqParam *)take(sizeof(UqParam));
    b.part = (uint32_t *)take((size_t)(pl.np + 1) * 4);
    b.counts = (uint32_t *)take((size_t)pl.E * 4);
    b.group = group;
    hipStream_t st = ctx->stream;

    // the corner points: measured, or known from the scaling of S
    if (!xmin) SUBKM_TRY(minmax_impl(ctx, S, n, d, b.mins, b.maxs, b.flag));
    hipLaunchKernelGGL(k_uq_prep, dim3(1), dim3(kUT), 0, st, b.mins, b.maxs, xmin, xmax, d, b.Ld,
                       b.Dd, b.Lf, b.Df, (int)metric, b.prm);
    SUBKM_LAUNCHED(ctx);
    if (landmarks) {
        const int64_t total = m * d;
        const int grid = (int)std::min<int64_t>(ceil_div(total, kUT), 4096);
        hipLaunchKernelGGL(k_uq_landmarks, dim3(grid), dim3(kUT), 0, st, b.Ld, b.Dd, d, m,
                           landmarks);
        SUBKM_LAUNCHED(ctx);
    }
    const bool v4 = (d % 4) == 0 && ((uintptr_t)S % 16) == 0 && ((uintptr_t)P % 16) == 0;
    const size_t lds = (size_t)m * sizeof(uint32_t);
    {
        const int kind = !v4 ? 0 : d <= 32 ? 8 : d <= 64 ? 16 : d <= 128 ? 32 : 1;
        auto launch = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3((unsigned)pl.nseg), dim3(kUT), lds, st, S, n, d, (int)m,
                               pl.seg, pl.nseg, b.Ld, b.Dd, b.Lf, b.Df, b.prm, group, b.counts);
        };
        if (metric == 0) switch (kind) {
                case 0: launch(k_uq_assign<0, 0>); break;
                case 8: launch(k_uq_assign<8, 0>); break;
                case 16: launch(k_uq_assign<16, 0>); break;
                case 32: launch(k_uq_assign<32, 0>); break;
                default: launch(k_uq_assign<1, 0>); break;
            }
        else switch (kind) {
                case 0: launch(k_uq_assign<0, 1>); break;
                case 8: launch(k_uq_assign<8, 1>); break;
                case 16: launch(k_uq_assign<16, 1>); break;
                case 32: launch(k_uq_assign<32, 1>); break;
                default: launch(k_uq_assign<1, 1>); break;
            }
        SUBKM_LAUNCHED(ctx);
    }
    hipLaunchKernelGGL(k_uq_scan_blocks, dim3(pl.np), dim3(kUT), 0, st, b.counts, pl.E, b.part);
    SUBKM_LAUNCHED(ctx);
    int nbits = 0;
    while ((1ll << nbits) < m) ++nbits;
    if (v4)
        hipLaunchKernelGGL(k_uq_scatter<4>, dim3((unsigned)pl.nseg), dim3(kUT), lds, st, S, n, d,
                           (int)m, nbits, pl.seg, pl.nseg, group, b.counts, b.part, pl.np, P,
                           perm, offsets);
    else
        hipLaunchKernelGGL(k_uq_scatter<1>, dim3((unsigned)pl.nseg), dim3(kUT), lds, st, S, n, d,
                           (int)m, nbits, pl.seg, pl.nseg, group, b.counts, b.part, pl.np, P,
                           perm, offsets);
    SUBKM_LAUNCHED(ctx);
    return SUBKM_OK;
}

// Local outputs of the groups: runs were launched for the non-empty groups
// only (run r is group gid[r]); empty groups get 0 moves and 0 objective.
__global__ __launch_bounds__(kUT) void k_uq_zero(int64_t T, int32_t *__restrict__ it,
                                                 double *__restrict__ sse) {
    const int64_t e = (int64_t)blockIdx.x * kUT + threadIdx.x;
    if (e < T) {
        it[e] = 0;
        sse[e] = 0.0;
    }
}

__global__ __launch_bounds__(kUT) void k_uq_put(const int32_t *__restrict__ gid, int R,
                                                const int32_t *__restrict__ it_c,
                                                const double *__restrict__ sse_c,
                                                int32_t *__restrict__ it,
                                                double *__restrict__ sse) {
    const int r = blockIdx.x * kUT + threadIdx.x;
    if (r < R) {
        it[gid[r]] = it_c[r];
        sse[gid[r]] = sse_c[r];
    }
}

subkm_status unequal_expand_local(subkm_ctx *ctx, const int32_t *gid, int R,
                                  const int32_t *it_c, const double *sse_c, int64_t T,
                                  int32_t *it, double *sse) {
    hipStream_t st = ctx->stream;
    hipLaunchKernelGGL(k_uq_zero, dim3((unsigned)ceil_div(T, kUT)), dim3(kUT), 0, st, T, it, sse);
    SUBKM_LAUNCHED(ctx);
    if (R > 0) {
        hipLaunchKernelGGL(k_uq_put, dim3((unsigned)ceil_div(R, kUT)), dim3(kUT), 0, st, gid, R,
                           it_c, sse_c, it, sse);
        SUBKM_LAUNCHED(ctx);
    }
    return SUBKM_OK;
}
