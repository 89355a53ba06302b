// Lloyd's k-means for runs whose centers do not fit on chip (Sec. II
// Algorithm 1 step 4 for large subclusters, Sec. V for the final run).
//
// Assignment with split-bfloat16 products (precision SUBKM_PREC_BF16).
//   Every run is centered on the midpoint m of its bounding box.  Before each
//   assignment the centers are turned into matrix-core fragments of
//   a = -2 (c - m) = a_hi + a_lo, both bfloat16 (a_hi = bf16(a),
//   a_lo = bf16(a - a_hi)); the points are split the same way in registers.
//   Three bfloat16 products a_hi x_hi + a_hi x_lo + a_lo x_hi, accumulated
//   in float32 on the matrix cores (v_mfma_f32_16x16x32_bf16) in two chains,
//   plus ||c - m||^2 and ||x - m||^2 give a float32 estimate D~ of
//   ||x - c||^2 whose error is below a bound E(x) (see split_bound).  A single
//   bfloat16 product would leave an error bound near 1% of ||x-m|| ||c-m||,
//   so large that almost every point of a dense run would need a recheck.
//
//   Every lane keeps the three smallest D~ of its centers.  The index of a
//   center rides in the 10 low mantissa bits of its value, so the minimum and
//   median instructions move it along for free; the perturbation (below
//   2^-13 |D~|) enters the bound.  Then, per point:
//     certain    the second smallest is provably larger than the smallest:
//                label = that center;
//     two-way    the third smallest is provably larger: binary64 distances to
//                the two candidates decide (lowest index on ties);
//     pooled     otherwise: the block collects such points, recomputes their
//                distances to all centers and keeps every center that cannot
//                be excluded, then compares those in binary64.
//   All binary64 distances use the arithmetic of the objective (attributes
//   left to right, separate multiply and add), so labels are those of exact
//   binary64 arithmetic on the float32 inputs, as in every other path.
//
// Update (every wide run, either precision).  Labels are counted per center,
// the counts scanned into starts, the points of the run ordered by label;
// then every center is the mean of its points, summed exactly as 64-bit
// fixed point (the same quantisation as the on-chip path), so centers do not
// depend on the order of the work.  A center without points stays.  The
// largest Euclidean move of the run decides convergence (strictly below tol).
#include "lloyd_dev.h"

#include <algorithm>
#include <cmath>

#pragma clang fp contract(off)

namespace subkm_lloyd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr float kPadNorm = 1.0e36f;  // ||c - m||^2 given to the padding rows of the last tile
constexpr float kBig = 3.0e38f;      // initial tracked value
constexpr uint32_t kIdxBits = 0x3FFu;  // center index bits of a tracked value (k <= 1024)
constexpr int kCandCap = 512;          // candidates per pooled round (16 points)
constexpr float kMaxNorm = 1.0e15f;    // ||x - m||, ||c - m|| beyond this: full binary64 scan

__device__ __forceinline__ uint32_t bf16_bits(float a) {
    const uint32_t u = __float_as_uint(a);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;  // round to nearest even
}

// a = hi + lo + r with hi = bf16(a), lo = bf16(a - hi), |r| <= 2^-16 |a|;
// a - hi is exact in float32 (hi holds the leading bits of a)
__device__ __forceinline__ void split_bf16(float a, uint32_t &h, uint32_t &l) {
    h = bf16_bits(a);
    l = bf16_bits(a - __uint_as_float(h << 16));
}

__device__ __forceinline__ bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ float fmin3(float a, float b) {
    return __builtin_amdgcn_fmed3f(a, b, -3.402823466e38f);
}
__device__ __forceinline__ float fmax3(float a, float b) {
    return __builtin_amdgcn_fmed3f(a, b, 3.402823466e38f);
}

// keep the three smallest of (b1 <= b2 <= b3) and e (all distinct)
__device__ __forceinline__ void top3_insert(float &b1, float &b2, float &b3, float e) {
    b3 = __builtin_amdgcn_fmed3f(b2, b3, fmax3(b1, e));
    b2 = __builtin_amdgcn_fmed3f(b1, b2, e);
    b1 = fmin3(b1, e);
}

__device__ __forceinline__ float encode(float v, uint32_t idx) {
    return __uint_as_float((__float_as_uint(v) & ~kIdxBits) | idx);
}

// Bounds of the value before the index was put into it: D~ lies in
// [lo_of(e), hi_of(e)] (|e - D~| < 2^-13 |D~|, plus the subnormal range).
__device__ __forceinline__ double lo_of(float e) {
    const double v = e;
    return v - 0x1p-12 * fabs(v) - 1e-38;
}
__device__ __forceinline__ double hi_of(float e) {
    const double v = e;
    return v + 0x1p-12 * fabs(v) + 1e-38;
}

// Error bound of one D~ for a point with ||x^ - m|| <= rx against centers
// with ||c^ - m|| <= rc (x^, c^ the float32 centered values), for S steps of
// 32 attributes (Dp = 32 S products per chain pass):
//   split      a x - (a_hi x_hi + a_hi x_lo + a_lo x_hi), summed over the
//              attributes: <= 2 (3 ub^2 + 2 ub^3) rx rc
//   chain 1    ||c - m||^2 + a_hi . x_hi, Dp additions in any order with
//              any faithful rounding (u' = 2^-23): gamma'_Dp (rc^2 (1+u) +
//              2 (1+ub)^2 rx rc)
//   chain 2    a_hi . x_lo + a_lo . x_hi: gamma'_2Dp 4 ub (1+ub) rx rc
//   combining  two float32 additions: 2 u' 1.05 (rx + rc)^2
//   centering  x^ = fl(x - m), c^ = fl(c - m): 2 u 1.02 (rx + rc)^2
//   norm       ||c^||^2 rounded once to float32: 1.01 u rc^2
// plus 1e-12 (rx + rc)^2 for the binary64 arithmetic that decides, and an
// absolute term for the subnormal range.  Products of bfloat16 values are
// exact in float32.
__device__ __forceinline__ double split_bound(int S, double rx, double rc) {
    const double u = 0x1p-24, u2 = 0x1p-23, ub = 0x1p-8;
    const double dp = 32.0 * S;
    const double g1 = dp * u2 / (1.0 - dp * u2), g2 = 2.0 * dp * u2 / (1.0 - 2.0 * dp * u2);
    const double cA = 2.0 * (3.0 * ub * ub + 2.0 * ub * ub * ub) + g1 * 2.0 * (1.0 + ub) * (1.0 + ub) +
                      g2 * 4.0 * ub * (1.0 + ub);
    const double cC = g1 * (1.0 + u) + 1.01 * u;
    const double cB = 2.0 * u2 * 1.05 + 2.0 * u * 1.02 + 1e-12;
    const double s = rx + rc;
    return cA * rx * rc + cC * rc * rc + cB * s * s + 1e-30;
}

// ---------------------------------------------------------------------------
// Center fragments.  For tile t (centers 16t .. 16t+15), step s (attributes
// 32s .. 32s+31) and part p (0 hi, 1 lo), lane l of the 64-lane fragment
// holds center 16t + l % 16, attributes 32s + 8 (l / 16) + j, j = 0..7, as
// eight bfloat16 values: the A operand of v_mfma_f32_16x16x32_bf16.
__global__ __launch_bounds__(256) void k_split_prep(const DevRun *__restrict__ runs, int r0,
                                                   const float *__restrict__ C,
                                                   const uint32_t *__restrict__ boxes, uint4 *frags,
                                                   float *cnorm, RunState *rstate) {
    __shared__ double s_red[256];
    const int r = r0 + blockIdx.y;
    const DevRun R = runs[r];
    if (!R.split) return;
    RunState *rs = rstate + r;
    if (rs->phase == PH_DONE) return;
    const int d = R.d, k = R.k;
    const int S = (d + 31) / 32;
    const int KT = (k + 15) / 16;
    const uint32_t *box = boxes + R.box_off;
    const float *Cr = C + R.c_off;
    double mx = 0.0;
    // one thread per (tile t, lane l): center 16t + l % 16, attributes
    // 32s + 8 (l / 16) + j of every step s; a wavefront covers one tile, so
    // the four lanes of a center finish its squared norm with two exchanges
    // (a fixed order: the result does not depend on the launch)
    const int64_t step = (int64_t)gridDim.x * 256;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)KT * 64; e += step) {
        const int l = (int)(e & 63);
        const int64_t t = e >> 6;
        const int64_t c = t * 16 + (l & 15);
        double a2 = 0.0;
        for (int s = 0; s < S; ++s) {
            const int j0 = 32 * s + 8 * (l >> 4);
            uint32_t hb[8], lb[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int dim = j0 + j;
                float a = 0.0f;
                if (c < k && dim < d) {
                    const float cp = Cr[c * d + dim] - box_mid(box, d, dim);
                    a2 = a2 + (double)cp * (double)cp;
                    a = -2.0f * cp;
                }
                split_bf16(a, hb[j], lb[j]);
            }
            uint4 H, L;
            H.x = hb[0] | (hb[1] << 16);
            H.y = hb[2] | (hb[3] << 16);
            H.z = hb[4] | (hb[5] << 16);
            H.w = hb[6] | (hb[7] << 16);
            L.x = lb[0] | (lb[1] << 16);
            L.y = lb[2] | (lb[3] << 16);
            L.z = lb[4] | (lb[5] << 16);
            L.w = lb[6] | (lb[7] << 16);
            const int64_t ts = t * S + s;
            frags[R.frag_off + (ts * 2 + 0) * 64 + l] = H;
            frags[R.frag_off + (ts * 2 + 1) * 64 + l] = L;
        }
        a2 = a2 + __shfl_xor(a2, 16, 64);
        a2 = a2 + __shfl_xor(a2, 32, 64);
        if (l < 16) {
            cnorm[R.cn_off + c] = c < k ? (float)a2 : kPadNorm;
            if (c < k) mx = fmax(mx, a2);
        }
    }
    mx = block_max(mx, s_red);
    if (threadIdx.x == 0 && mx > 0.0)
        atomicMax(&rs->rc2_bits, (unsigned long long)__double_as_longlong(mx));
}

// B-operand fragments of one point (lane: column l % 16, attributes
// 32s + 8 (l / 16) + j) and its partial ||x^ - m||^2 over those attributes.
template <int S>
__device__ __forceinline__ void point_frags(const float *X, int64_t p, bool ok, int d,
                                            const float (&mq)[S][8], int kk, u32x4 (&xh)[S],
                                            u32x4 (&xl)[S], float &s2) {
    s2 = 0.0f;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        uint32_t hb[8], lb[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int dim = 32 * s + 8 * kk + j;
            const bool in = ok && dim < d;
            const float xv = in ? X[p * d + dim] : 0.0f;
            const float v = in ? xv - mq[s][j] : 0.0f;
            s2 = __builtin_fmaf(v, v, s2);
            split_bf16(v, hb[j], lb[j]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            xh[s][q] = hb[2 * q] | (hb[2 * q + 1] << 16);
            xl[s][q] = lb[2 * q] | (lb[2 * q + 1] << 16);
        }
    }
}

// D~ of the 4 centers (rows 4 (l/16) + r of tile t) against this lane's point
template <int S>
__device__ __forceinline__ floatx4 split_tile(const u32x4 (&ah)[S], const u32x4 (&al)[S],
                                              floatx4 cn4, const u32x4 (&xh)[S],
                                              const u32x4 (&xl)[S], float xn2) {
    floatx4 a1 = cn4;
    floatx4 a2 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < S; ++s)
        a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ah[s]), as_bf(xh[s]), a1, 0, 0, 0);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        a2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ah[s]), as_bf(xl[s]), a2, 0, 0, 0);
        a2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(al[s]), as_bf(xh[s]), a2, 0, 0, 0);
    }
    floatx4 v;
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = (a1[r] + a2[r]) + xn2;
    return v;
}

template <int S>
__device__ __forceinline__ void load_center_tile(const uint4 *F, const float *cnr, int t, int lane,
                                                 int kk, u32x4 (&ah)[S], u32x4 (&al)[S],
                                                 floatx4 &cn4) {
    const u32x4 *Ft = reinterpret_cast<const u32x4 *>(F) + (int64_t)t * S * 128;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        ah[s] = Ft[(s * 2 + 0) * 64 + lane];
        al[s] = Ft[(s * 2 + 1) * 64 + lane];
    }
    cn4 = *reinterpret_cast<const floatx4 *>(cnr + t * 16 + 4 * kk);
}

// one center tile against the wavefront's four 16-point groups: every lane
// inserts its four tagged values per group into the group's top three
template <int S>
__device__ __forceinline__ void track_tile(const u32x4 (&ah)[S], const u32x4 (&al)[S], floatx4 cn4,
                                           uint32_t cbase, const u32x4 (&xh)[4][S],
                                           const u32x4 (&xl)[4][S], const float (&xn2)[4],
                                           float (&b1)[4], float (&b2)[4], float (&b3)[4]) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const floatx4 v = split_tile<S>(ah, al, cn4, xh[g], xl[g], xn2[g]);
#pragma unroll
        for (int r = 0; r < 4; ++r) top3_insert(b1[g], b2[g], b3[g], encode(v[r], cbase + r));
    }
}

constexpr int kChunkTiles = 2;  // center tiles per staged chunk

typedef __attribute__((address_space(3))) void lds_void;

// Copy the fragments of center tiles [t0, t0 + nt) (contiguous in memory)
// into LDS with direct global-to-LDS loads: one 1 KiB fragment per
// instruction and wavefront, no registers involved.
template <int S>
__device__ __forceinline__ void stage_chunk(const uint4 *F, int t0, int nt, uint4 *buf, int wave,
                                            int lane) {
    const uint4 *src = F + (int64_t)t0 * S * 128;
    for (int f = wave; f < nt * S * 2; f += kAT / 64)
        __builtin_amdgcn_global_load_lds((const void *)(src + f * 64 + lane), (lds_void *)(buf + f * 64), 16, 0, 0);
}

// One staged center tile against the wavefront's four 16-point groups; the
// products are accumulated in the same order as split_tile.
template <int S>
__device__ __forceinline__ void track_tile_lds(const uint4 *tb, int lane, floatx4 cn4, uint32_t cbase,
                                               const u32x4 (&xh)[4][S], const u32x4 (&xl)[4][S],
                                               const float (&xn2)[4], float (&b1)[4], float (&b2)[4],
                                               float (&b3)[4]) {
    floatx4 a1[4], a2[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        a1[g] = cn4;
        a2[g] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    const u32x4 *t4 = reinterpret_cast<const u32x4 *>(tb);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const u32x4 ah = t4[(s * 2 + 0) * 64 + lane];
        const u32x4 al = t4[(s * 2 + 1) * 64 + lane];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            a1[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ah), as_bf(xh[g][s]), a1[g], 0, 0, 0);
            a2[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ah), as_bf(xl[g][s]), a2[g], 0, 0, 0);
            a2[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(al), as_bf(xh[g][s]), a2[g], 0, 0, 0);
        }
    }
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            top3_insert(b1[g], b2[g], b3[g], encode((a1[g][r] + a2[g][r]) + xn2[g], cbase + r));
}

enum : int32_t { ST_CERTAIN = 0, ST_TWO = 1, ST_POOL = 2, ST_FULL = 3 };

// Assignment of one tile of kAT points of a split run: four wavefronts of 64
// points, each point's fragments held in registers while all center tiles
// stream through (fragments read straight from memory, the next tile's while
// the current one computes).
template <int S>
__global__ __launch_bounds__(kAT, 2) void k_assign_split(
    const float *__restrict__ P, const DevRun *__restrict__ runs, const Item *__restrict__ items,
    int item_base, const float *__restrict__ C, const uint4 *__restrict__ frags,
    const float *__restrict__ cnorm, int32_t *labels, RunState *rstate, double *objpart,
    const uint32_t *__restrict__ boxes, int last_pass) {
    __shared__ int32_t s_c1[kAT], s_c2[kAT], s_st[kAT], s_lab[kAT];
    __shared__ float s_thr[kAT];
    __shared__ int32_t s_pool[kAT];
    __shared__ uint32_t s_npool, s_ncand;
    __shared__ int32_t s_cq[kCandCap], s_cc[kCandCap];
    __shared__ double s_cd[kCandCap];
    __shared__ double s_red[kAT];
    __shared__ uint4 s_fa[kChunkTiles * S * 128], s_fb[kChunkTiles * S * 128];

    const Item itm = items[item_base + blockIdx.x];
    const DevRun R = runs[itm.run];
    RunState *rs = rstate + itm.run;
    const int32_t ph = rs->phase;
    if (ph == PH_DONE) return;
    const bool want_obj = last_pass || ph == PH_FINAL;
    const int d = R.d, k = R.k, KT = (k + 15) / 16;
    const float *X = P + R.x_off;
    const float *Cr = C + R.c_off;
    const uint32_t *box = boxes + R.box_off;
    const uint4 *F = frags + R.frag_off;
    const float *cnr = cnorm + R.cn_off;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kk = lane >> 4;
    const int64_t first_w = itm.first + wave * 64;
    if (threadIdx.x == 0) s_npool = 0;

    float mq[S][8];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int dim = 32 * s + 8 * kk + j;
            mq[s][j] = dim < d ? box_mid(box, d, dim) : 0.0f;
        }

    u32x4 xh[4][S], xl[4][S];
    float xn2[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int64_t p = first_w + g * 16 + col;
        float s2;
        point_frags<S>(X, p, p < R.n, d, mq, kk, xh[g], xl[g], s2);
        s2 += __shfl_xor(s2, 16, 64);
        s2 += __shfl_xor(s2, 32, 64);
        xn2[g] = s2;
    }

    float b1[4], b2[4], b3[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) b1[g] = b2[g] = b3[g] = kBig;

    // center fragments stream through two LDS buffers of kChunkTiles tiles:
    // the next chunk is copied in while the current one computes
    const int nch = (KT + kChunkTiles - 1) / kChunkTiles;
    stage_chunk<S>(F, 0, min(kChunkTiles, KT), s_fa, wave, lane);
    floatx4 cn4 = *reinterpret_cast<const floatx4 *>(cnr + 4 * kk);
    for (int ch = 0; ch < nch; ++ch) {
        uint4 *cur = (ch & 1) ? s_fb : s_fa;
        uint4 *nxt = (ch & 1) ? s_fa : s_fb;
        __builtin_amdgcn_s_waitcnt(0);  // this wavefront's copies of chunk ch are done
        __syncthreads();                // everyone's; and nobody still reads nxt
        const int t0 = ch * kChunkTiles;
        const int nt = min(kChunkTiles, KT - t0);
        if (ch + 1 < nch) stage_chunk<S>(F, t0 + kChunkTiles, min(kChunkTiles, KT - t0 - kChunkTiles), nxt, wave, lane);
        for (int tt = 0; tt < nt; ++tt) {
            const int t = t0 + tt;
            const floatx4 cnn = t + 1 < KT ? *reinterpret_cast<const floatx4 *>(cnr + (t + 1) * 16 + 4 * kk) : cn4;
            track_tile_lds<S>(cur + tt * S * 128, lane, cn4, (uint32_t)(t * 16 + 4 * kk), xh, xl, xn2, b1, b2, b3);
            cn4 = cnn;
        }
    }

    // the four lanes of a point hold disjoint center sets: merge their triples
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int o = 16; o <= 32; o <<= 1) {
            const float o1 = __shfl_xor(b1[g], o, 64);
            const float o2 = __shfl_xor(b2[g], o, 64);
            const float o3 = __shfl_xor(b3[g], o, 64);
            top3_insert(b1[g], b2[g], b3[g], o1);
            top3_insert(b1[g], b2[g], b3[g], o2);
            top3_insert(b1[g], b2[g], b3[g], o3);
        }

    const double rc2 = __longlong_as_double((long long)rs->rc2_bits);
    const double rc = sqrt(rc2) * (1.0 + 1e-12);
    if (kk == 0) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const double rx = sqrt((double)xn2[g]) * (1.0 + 0x1p-14);
            const double E = split_bound(S, rx, rc);
            const int32_t c1 = (int32_t)(__float_as_uint(b1[g]) & kIdxBits);
            const int32_t c2 = (int32_t)(__float_as_uint(b2[g]) & kIdxBits);
            const double top = hi_of(b1[g]) + 2.0 * E;
            int32_t st;
            if (!(rx < kMaxNorm && rc < kMaxNorm) || c1 >= k) st = ST_FULL;
            else if (k == 1 || lo_of(b2[g]) > top) st = ST_CERTAIN;
            else if (lo_of(b3[g]) > top && c2 < k) st = ST_TWO;
            else st = ST_POOL;
            // pooled points keep every center whose tracked value could lie
            // below top: e <= lo_of^-1(top), rounded up
            const double thr = top >= 0.0 ? (top + 1e-38) / (1.0 - 0x1p-12) : (top + 1e-38) / (1.0 + 0x1p-12);
            const int slot = wave * 64 + g * 16 + col;
            s_c1[slot] = c1;
            s_c2[slot] = c2;
            s_st[slot] = st;
            s_thr[slot] = (float)(thr + 0x1p-20 * fabs(thr) + 1e-37);
        }
    }
    __syncthreads();  // LDS results of every wavefront (and s_npool = 0) visible

    const int my = threadIdx.x;
    const int64_t i = itm.first + my;
    const bool valid = i < R.n;
    const float *xg = X + (valid ? i : 0) * d;
    int32_t st = valid ? s_st[my] : ST_CERTAIN;
    int32_t lab = s_c1[my];
    double obj = 0.0;
    bool have_obj = false;
    if (st == ST_TWO) {
        const int32_t c2 = s_c2[my];
        double d1 = dist64(xg, Cr + (int64_t)lab * d, d);
        const double d2 = dist64(xg, Cr + (int64_t)c2 * d, d);
        if (d2 < d1 || (d2 == d1 && c2 < lab)) {
            lab = c2;
            d1 = d2;
        }
        obj = d1;
        have_obj = true;
    } else if (st == ST_POOL) {
        s_pool[atomicAdd(&s_npool, 1u)] = my;
    }
    // full scans: one wavefront per point
    {
        unsigned long long todo = __ballot(st == ST_FULL);
        while (todo) {
            const int t = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int32_t w = wave_argmin64(X + (first_w + t) * d, Cr, d, k);
            if (lane == t) lab = w;
        }
    }
    __syncthreads();
    const int np = (int)s_npool;
    for (int q0 = 0; q0 < np; q0 += 16) {
        const int nq = np - q0 < 16 ? np - q0 : 16;
        if (threadIdx.x == 0) s_ncand = 0;
        __syncthreads();
        {
            // every wavefront rebuilds the fragments of the (up to) 16 pooled
            // points and scans its share of the center tiles
            const bool okq = col < nq;
            const int pl = s_pool[q0 + (okq ? col : 0)];
            u32x4 yh[S], yl[S];
            float y2;
            point_frags<S>(X, itm.first + pl, true, d, mq, kk, yh, yl, y2);
            y2 += __shfl_xor(y2, 16, 64);
            y2 += __shfl_xor(y2, 32, 64);
            const float thr = okq ? s_thr[pl] : -kBig;
            for (int t = wave; t < KT; t += kAT / 64) {
                u32x4 ch[S], cl[S];
                floatx4 cn4;
                load_center_tile<S>(F, cnr, t, lane, kk, ch, cl, cn4);
                const floatx4 v = split_tile<S>(ch, cl, cn4, yh, yl, y2);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = t * 16 + 4 * kk + r;
                    if (c < k && encode(v[r], (uint32_t)c) <= thr) {
                        const uint32_t q = atomicAdd(&s_ncand, 1u);
                        if (q < (uint32_t)kCandCap) {
                            s_cq[q] = col;
                            s_cc[q] = c;
                        }
                    }
                }
            }
        }
        __syncthreads();
        const uint32_t ncand = s_ncand;
        if (ncand <= (uint32_t)kCandCap) {
            for (uint32_t e = threadIdx.x; e < ncand; e += kAT) {
                const int pl = s_pool[q0 + s_cq[e]];
                s_cd[e] = dist64(X + (itm.first + pl) * d, Cr + (int64_t)s_cc[e] * d, d);
            }
            __syncthreads();
            if ((int)threadIdx.x < nq) {
                double best = INFINITY;
                int32_t bi = 0x7fffffff;
                for (uint32_t e = 0; e < ncand; ++e)
                    if (s_cq[e] == (int)threadIdx.x) {
                        const double v = s_cd[e];
                        if (v < best || (v == best && s_cc[e] < bi)) {
                            best = v;
                            bi = s_cc[e];
                        }
                    }
                s_lab[s_pool[q0 + threadIdx.x]] = bi;
            }
        } else {
            // too many candidates (not expected): full scans of this round
            for (int q = wave; q < nq; q += kAT / 64) {
                const int pl = s_pool[q0 + q];
                const int32_t w = wave_argmin64(X + (itm.first + pl) * d, Cr, d, k);
                if (lane == 0) s_lab[pl] = w;
            }
        }
        __syncthreads();
    }
    if (st == ST_POOL) lab = s_lab[my];
    if (valid) {
        labels[R.lab_off + i] = lab;
        if (want_obj && !have_obj) obj = dist64(xg, Cr + (int64_t)lab * d, d);
    }
    const unsigned long long nre = __popcll(__ballot(valid && st != ST_CERTAIN));
    if (lane == 0 && nre) atomicAdd(&rs->rechecks, nre);
    if (want_obj) {
        const double tot = block_sum_det(obj, s_red);
        if (threadIdx.x == 0) objpart[item_base + blockIdx.x] = tot;
    }
}

// ---------------------------------------------------------------------------
// Update of the wide runs.  cnt holds per run (at cnt_off) counts[k],
// starts[k] and cursors[k] (the counts are added by k_wcount);
// order holds per run (at lab_off) the run's point indices grouped by
// label.
// exclusive scan of the counts of run r0 + blockIdx.x into starts and cursors
__global__ __launch_bounds__(kAT) void k_wscan(const DevRun *__restrict__ runs, int r0,
                                              const RunState *__restrict__ rstate, int32_t *cnt) {
    __shared__ int32_t s_v[kAT];
    const int r = r0 + blockIdx.x;
    const DevRun R = runs[r];
    if (R.fused || rstate[r].phase != PH_ITER) return;
    int32_t *counts = cnt + R.cnt_off;
    int32_t *starts = counts + R.k;
    int32_t *cursor = starts + R.k;
    int32_t carry = 0;
    for (int c0 = 0; c0 < R.k; c0 += kAT) {
        const int c = c0 + threadIdx.x;
        const int32_t v = c < R.k ? counts[c] : 0;
        s_v[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kAT; o <<= 1) {
            const int32_t a = threadIdx.x >= (unsigned)o ? s_v[threadIdx.x - o] : 0;
            __syncthreads();
            s_v[threadIdx.x] += a;
            __syncthreads();
        }
        const int32_t incl = s_v[threadIdx.x];
        if (c < R.k) {
            starts[c] = carry + incl - v;
            cursor[c] = carry + incl - v;
        }
        carry += s_v[kAT - 1];
        __syncthreads();
    }
}

// Counting and placement by label work on chunks of up to kChunkItems
// assignment items (consecutive points; a chunk is cut where the run
// changes).  Runs with k <= kHistK aggregate in an LDS histogram and touch
// each global counter once per chunk; larger runs aggregate per wavefront.
constexpr int kChunkItems = 16;
constexpr int kHistK = 4096;

// Visits the same-run segments of block blockIdx.x's chunk of items
// [i0, i0 + ni): f(R, run, first item, end item) for runs still iterating.
template <class F>
__device__ __forceinline__ void for_chunk_segments(const DevRun *__restrict__ runs,
                                                   const Item *__restrict__ items, int i0, int ni,
                                                   const RunState *__restrict__ rstate, F &&f) {
    const int a = i0 + blockIdx.x * kChunkItems;
    const int b = min(i0 + ni, a + kChunkItems);
    for (int it = a; it < b;) {
        const int run = items[it].run;
        const DevRun R = runs[run];
        const int e = min(b, R.item0 + R.nitems);
        if (rstate[run].phase == PH_ITER) f(R, run, it, e);
        it = e;
    }
}

// counts[c] = points labelled c (k_wfin zeroes them after the update)
__global__ __launch_bounds__(kAT) void k_wcount(const DevRun *__restrict__ runs,
                                               const Item *__restrict__ items, int i0, int ni,
                                               const int32_t *__restrict__ labels,
                                               const RunState *__restrict__ rstate,
                                               int32_t *cnt) {
    __shared__ int32_t h[kHistK];
    for_chunk_segments(runs, items, i0, ni, rstate, [&](const DevRun &R, int, int a, int e) {
        int32_t *counts = cnt + R.cnt_off;
        const bool lds = R.k <= kHistK;
        if (lds) {
            for (int c = threadIdx.x; c < R.k; c += kAT) h[c] = 0;
            __syncthreads();
        }
        for (int it = a; it < e; ++it) {
            const int64_t i = items[it].first + threadIdx.x;
            const int32_t l = i < R.n ? labels[R.lab_off + i] : -1;
            const bool valid = (uint32_t)l < (uint32_t)R.k;
            if (lds) {
                if (valid) atomicAdd(&h[l], 1);
            } else {
                wave_count_add(counts, valid, l, label_bits(R.k));
            }
        }
        if (lds) {
            __syncthreads();
            for (int c = threadIdx.x; c < R.k; c += kAT)
                if (h[c]) atomicAdd(&counts[c], h[c]);
            __syncthreads();
        }
    });
}

// order[starts[c] ..) = the points labelled c (any order inside a center:
// the sums over them are exact integers), and their labels at olab_off
__global__ __launch_bounds__(kAT) void k_wscatter(const DevRun *__restrict__ runs,
                                                 const Item *__restrict__ items, int i0, int ni,
                                                 const int32_t *__restrict__ labels,
                                                 const RunState *__restrict__ rstate, int32_t *cnt,
                                                 int32_t *order, int64_t olab_off) {
    __shared__ int32_t h[kHistK];
    for_chunk_segments(runs, items, i0, ni, rstate, [&](const DevRun &R, int, int a, int e) {
        int32_t *cursor = cnt + R.cnt_off + 2 * (int64_t)R.k;
        const bool lds = R.k <= kHistK;
        if (lds) {
            // the segment's count per label, then one range per label
            for (int c = threadIdx.x; c < R.k; c += kAT) h[c] = 0;
            __syncthreads();
            for (int it = a; it < e; ++it) {
                const int64_t i = items[it].first + threadIdx.x;
                const int32_t l = i < R.n ? labels[R.lab_off + i] : -1;
                if ((uint32_t)l < (uint32_t)R.k) atomicAdd(&h[l], 1);
            }
            __syncthreads();
            for (int c = threadIdx.x; c < R.k; c += kAT)
                if (h[c]) h[c] = atomicAdd(&cursor[c], h[c]);
            __syncthreads();
        }
        for (int it = a; it < e; ++it) {
            const int64_t i = items[it].first + threadIdx.x;
            const int32_t l = i < R.n ? labels[R.lab_off + i] : -1;
            const bool valid = (uint32_t)l < (uint32_t)R.k;
            int32_t pos;
            if (lds) pos = valid ? atomicAdd(&h[l], 1) : 0;
            else pos = wave_count_add(cursor, valid, l, label_bits(R.k));
            if (valid && (int64_t)pos < R.n) {
                order[R.lab_off + pos] = (int32_t)i;
                order[olab_off + R.lab_off + pos] = l;
            }
        }
        if (lds) __syncthreads();
    });
}

// Balanced sums for runs with d <= kWalkD.  A wavefront holds R.wpp points
// side by side (g = 64 / R.wpp lanes per point, lane j0 of a group holding
// attributes j0 and j0 + g); each lane group walks its own window of kWalkW
// consecutive positions of the run's label-sorted order and keeps the running
// fixed-point sum of the current center.  Windows are aligned to kWalkW
// positions whatever g is.  A center whose points all lie in one window gets
// its new value right away; the partial sums of a center that crosses a
// window edge go to the run's int64 sums (exact, so the order of the atomic
// additions does not matter) and k_wfin finishes it.
__global__ __launch_bounds__(kAT) void k_wwalk(const float *__restrict__ P,
                                              const DevRun *__restrict__ runs,
                                              const Item *__restrict__ items, int w0,
                                              const int32_t *__restrict__ order, int64_t olab_off,
                                              float *C, RunState *rstate,
                                              const int32_t *__restrict__ cnt, long long *gsum) {
    constexpr int kU = 8;
    const Item itm = items[w0 + blockIdx.x];
    const DevRun R = runs[itm.run];
    RunState *rs = rstate + itm.run;
    if (rs->phase != PH_ITER || R.d > kWalkD) return;
    const int d = R.d;
    const int s = fix_shift_of(rs->absmax_bits);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ppw = R.wpp, g = 64 / ppw, sub = lane / g, j0 = lane % g;
    const int ja = j0, jc = j0 + g;
    const int64_t a = (int64_t)itm.first + ((int64_t)wave * ppw + sub) * kWalkW;
    const int64_t b = min(R.n, a + kWalkW);
    const int nb = (int)max((int64_t)0, b - a);  // positions of this lane's group
    const int32_t *counts = cnt + R.cnt_off;
    const int32_t *starts = counts + R.k;
    const float *X = P + R.x_off;
    const int32_t *ord = order + R.lab_off;
    const int32_t *olab = order + olab_off + R.lab_off;
    float *Cr = C + R.c_off;
    long long *gs = gsum + R.sum_off;
    double wmax = 0.0;
    int32_t cur = -1;
    long long A0 = 0, A1 = 0;
    // every lane of a group takes the same branches (cur is the group's):
    // the exchanges below stay inside the group
    auto flush = [&]() {
        if (cur < 0) return;
        const int32_t st = starts[cur], n_c = counts[cur];
        if (st >= a && (int64_t)st + n_c <= b) {
            double dv2 = 0.0;
            if (ja < d) {
                const float old = Cr[(int64_t)cur * d + ja];
                const double nv = ldexp((double)A0, -s) / (double)n_c;
                const double dv = nv - (double)old;
                dv2 = dv * dv;
                Cr[(int64_t)cur * d + ja] = (float)nv;
            }
            if (jc < d) {
                const float old = Cr[(int64_t)cur * d + jc];
                const double nv = ldexp((double)A1, -s) / (double)n_c;
                const double dv = nv - (double)old;
                dv2 = dv2 + dv * dv;
                Cr[(int64_t)cur * d + jc] = (float)nv;
            }
            for (int o = g >> 1; o > 0; o >>= 1) dv2 = dv2 + __shfl_xor(dv2, o, 64);
            wmax = fmax(wmax, sqrt(dv2));
        } else {
            if (ja < d) atomicAdd((unsigned long long *)&gs[(int64_t)cur * d + ja], (unsigned long long)A0);
            if (jc < d) atomicAdd((unsigned long long *)&gs[(int64_t)cur * d + jc], (unsigned long long)A1);
        }
    };
    // positions are read g at a time per group (lane j0 reads position
    // q0 + j0) and broadcast inside the group, kU rows in flight per lane;
    // the trip counts are the same for every lane of the wavefront
    for (int q0 = 0; q0 < kWalkW; q0 += g) {
        const bool okp = q0 + j0 < nb;
        const int32_t myp = okp ? ord[a + q0 + j0] : 0;
        const int32_t myl = okp ? olab[a + q0 + j0] : -1;
        for (int ub = 0; ub < g; ub += kU) {
            float v0[kU], v1[kU];
            int32_t lu[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int qq = ub + u < g ? ub + u : g - 1;
                const int64_t p = __shfl(myp, sub * g + qq, 64);
                lu[u] = __shfl(myl, sub * g + qq, 64);
                const bool ok = ub + u < g && q0 + ub + u < nb;
                v0[u] = (ok && ja < d) ? X[p * d + ja] : 0.0f;
                v1[u] = (ok && jc < d) ? X[p * d + jc] : 0.0f;
                if (!ok) lu[u] = -1;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                if (lu[u] >= 0) {  // the same for every lane of the group
                    if (lu[u] != cur) {
                        flush();
                        cur = lu[u];
                        A0 = 0;
                        A1 = 0;
                    }
                    A0 += to_fixed(v0[u], s);
                    A1 += to_fixed(v1[u], s);
                }
            }
        }
    }
    flush();
    for (int o = 32; o > 0; o >>= 1) wmax = fmax(wmax, __shfl_xor(wmax, o, 64));
    if (lane == 0 && wmax > 0.0)
        atomicMax(&rs->shift_bits, (unsigned long long)__double_as_longlong(wmax));
}

// New centers of update item (run, first center c0, kcu centers), one
// wavefront per center.  For d <= kWalkD only the centers that crossed a
// walk window are left: their sums are in gsum (zeroed again here).  For
// wider points the wavefront sums the center's points itself: lanes split
// the attributes, two per lane and pass (narrow points: several points side
// by side), the point indices are read 64 at a time and broadcast, and every
// lane keeps kU rows in flight.  The run's last item decides convergence.
__global__ __launch_bounds__(kAT) void k_wfin(const float *__restrict__ P,
                                             const DevRun *__restrict__ runs,
                                             const Item *__restrict__ items, int u0,
                                             const int32_t *__restrict__ order, float *C,
                                             RunState *rstate, int32_t *cnt, long long *gsum,
                                             double tol) {
    constexpr int kU = 8;
    __shared__ double s_red[kAT];
    __shared__ uint32_t s_last;
    const Item itm = items[u0 + blockIdx.x];
    const DevRun R = runs[itm.run];
    RunState *rs = rstate + itm.run;
    const int32_t ph = rs->phase;
    if (ph == PH_DONE) return;
    if (ph == PH_FINAL) {
        // the assignment that just ran was the last one of this run
        if (itm.first == 0 && threadIdx.x == 0) rs->phase = PH_DONE;
        return;
    }
    const int d = R.d;
    const int s = fix_shift_of(rs->absmax_bits);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int dg = 1;  // lanes per point: the next power of two >= d, at most 64
    while (dg < d && dg < 64) dg <<= 1;
    const int ppw = 64 / dg, sub = lane / dg, j0 = lane % dg;
    int32_t *counts = cnt + R.cnt_off;
    const int32_t *starts = counts + R.k;
    const float *X = P + R.x_off;
    const int32_t *ord = order + R.lab_off;
    float *Cr = C + R.c_off;
    const int c1 = min(R.k, itm.first + R.kcu);
    double mx = 0.0;
    const bool walked = d <= kWalkD;
    long long *gs = gsum + R.sum_off;
    if (walked && R.kcu == kWalkCenters) {
        // one center per lane: the counts are read (and cleared) 64 at a
        // time; the centers that crossed a walk window are finished one
        // after the other by the whole wavefront
        for (int cb = itm.first + wave * 64; cb < c1; cb += kAT) {
            const int c = cb + lane;
            const int32_t n_c = c < c1 ? counts[c] : 0;
            const int32_t st = c < c1 ? starts[c] : 0;
            if (c < c1) counts[c] = 0;
            unsigned long long todo = __ballot(n_c > 0 && st / kWalkW != (st + n_c - 1) / kWalkW);
            while (todo) {
                const int t = __ffsll(todo) - 1;
                todo &= todo - 1;
                const int ct = cb + t;
                const int32_t nt = __shfl(n_c, t, 64);
                double dv2 = 0.0;
                for (int j = lane; j < d; j += 64) {
                    const long long a = gs[(int64_t)ct * d + j];
                    gs[(int64_t)ct * d + j] = 0;
                    const float old = Cr[(int64_t)ct * d + j];
                    const double nv = ldexp((double)a, -s) / (double)nt;
                    const double dv = nv - (double)old;
                    dv2 = dv2 + dv * dv;
                    Cr[(int64_t)ct * d + j] = (float)nv;
                }
                for (int o = 32; o > 0; o >>= 1) dv2 = dv2 + __shfl_xor(dv2, o, 64);
                mx = fmax(mx, sqrt(dv2));
            }
        }
    }
    for (int c = itm.first + wave; R.kcu != kWalkCenters && c < c1; c += kAT / 64) {
        const int32_t n_c = counts[c];
        const int32_t st = starts[c];
        double mv2 = 0.0;
        if (walked) {
            // one wavefront per center; only centers that crossed a walk
            // window are left to finish
            if (n_c > 0 && st / kWalkW != (st + n_c - 1) / kWalkW) {
                double dv2 = 0.0;
                for (int j = lane; j < d; j += 64) {
                    const long long a = gs[(int64_t)c * d + j];
                    gs[(int64_t)c * d + j] = 0;
                    const float old = Cr[(int64_t)c * d + j];
                    const double nv = ldexp((double)a, -s) / (double)n_c;
                    const double dv = nv - (double)old;
                    dv2 = dv2 + dv * dv;
                    Cr[(int64_t)c * d + j] = (float)nv;
                }
                for (int o = 32; o > 0; o >>= 1) dv2 = dv2 + __shfl_xor(dv2, o, 64);
                mv2 = dv2;
            }
        } else if (n_c > 0) {
            for (int jb = 0; jb < d; jb += 2 * dg) {
                const int ja = jb + j0, jc = jb + j0 + dg;  // this lane's two attributes
                long long a0 = 0, a1 = 0;
                for (int m0 = 0; m0 < n_c; m0 += 64) {
                    const int nb = min(64, n_c - m0);
                    const int32_t myp = lane < nb ? ord[st + m0 + lane] : 0;
                    // the trip count is the same for every lane: the
                    // broadcasts read lanes that are all active
                    for (int qb = 0; qb < nb; qb += kU * ppw) {
                        float v0[kU], v1[kU];
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int qq = qb + sub + u * ppw;
                            const int64_t p = __shfl(myp, qq < 64 ? qq : 63, 64);
                            const bool ok = qq < nb;
                            v0[u] = (ok && ja < d) ? X[p * d + ja] : 0.0f;
                            v1[u] = (ok && jc < d) ? X[p * d + jc] : 0.0f;
                        }
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            a0 += to_fixed(v0[u], s);
                            a1 += to_fixed(v1[u], s);
                        }
                    }
                }
                for (int o = dg; o < 64; o <<= 1) {
                    a0 += __shfl_xor(a0, o, 64);
                    a1 += __shfl_xor(a1, o, 64);
                }
                double dv2 = 0.0;
                if (sub == 0) {
                    if (ja < d) {
                        const float old = Cr[(int64_t)c * d + ja];
                        const double nv = ldexp((double)a0, -s) / (double)n_c;
                        const double dv = nv - (double)old;
                        dv2 = dv * dv;
                        Cr[(int64_t)c * d + ja] = (float)nv;
                    }
                    if (jc < d) {
                        const float old = Cr[(int64_t)c * d + jc];
                        const double nv = ldexp((double)a1, -s) / (double)n_c;
                        const double dv = nv - (double)old;
                        dv2 = dv2 + dv * dv;
                        Cr[(int64_t)c * d + jc] = (float)nv;
                    }
                }
                // fixed-order tree over the lanes
                for (int o = 32; o > 0; o >>= 1) dv2 = dv2 + __shfl_xor(dv2, o, 64);
                mv2 = mv2 + dv2;
            }
        }
        if (lane == 0) counts[c] = 0;
        mx = fmax(mx, sqrt(mv2));
    }
    mx = block_max(mx, s_red);
    if (threadIdx.x == 0) {
        atomicMax(&rs->shift_bits, (unsigned long long)__double_as_longlong(mx));
        __threadfence();
        s_last = atomicAdd(&rs->ucount, 1u) == (uint32_t)R.nuitems - 1;
        if (s_last) {
            __threadfence();
            const unsigned long long sb =
                __hip_atomic_load(&rs->shift_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            rs->iters += 1;
            rs->phase = __longlong_as_double((long long)sb) < tol ? PH_FINAL : PH_ITER;
            rs->shift_bits = 0;
            rs->ucount = 0;
            rs->rc2_bits = 0;
        }
    }
}

template <int S>
subkm_status launch_split(subkm_ctx *ctx, int i0, int ni, const float *P, const DevRun *runs,
                          const Item *items, const float *C, const uint4 *frags,
                          const float *cnorm, int32_t *labels, RunState *rs, double *objpart,
                          const uint32_t *boxes, int last_pass) {
    hipLaunchKernelGGL(k_assign_split<S>, dim3(ni), dim3(kAT), 0, ctx->stream, P, runs, items, i0, C,
                       frags, cnorm, labels, rs, objpart, boxes, last_pass);
    SUBKM_LAUNCHED(ctx);
    return SUBKM_OK;
}

}  // namespace

subkm_status wide_split_prep(subkm_ctx *ctx, int r0, int nr, int kt_max, int steps_max,
                             const DevRun *runs, const float *C, const uint32_t *boxes,
                             uint4 *frags, float *cnorm, RunState *rs) {
    if (nr <= 0) return SUBKM_OK;
    ProfScope ps(ctx, PK_UPDATE);
    (void)steps_max;
    const int64_t work = (int64_t)kt_max * 64;
    const int bx = (int)std::min<int64_t>(ceil_div(work, 256), 1024);
    hipLaunchKernelGGL(k_split_prep, dim3(bx, nr), dim3(256), 0, ctx->stream, runs, r0, C, boxes,
                       frags, cnorm, rs);
    SUBKM_LAUNCHED(ctx);
    return SUBKM_OK;
}

subkm_status wide_assign_split(subkm_ctx *ctx, int S, int i0, int ni, const float *P,
                               const DevRun *runs, const Item *items, const float *C,
                               const uint4 *frags, const float *cnorm, int32_t *labels,
                               RunState *rs, double *objpart, const uint32_t *boxes,
                               int last_pass) {
    if (ni <= 0) return SUBKM_OK;
    ProfScope ps(ctx, PK_ASSIGN);
    switch (S) {
        case 1: return launch_split<1>(ctx, i0, ni, P, runs, items, C, frags, cnorm, labels, rs, objpart, boxes, last_pass);
        case 2: return launch_split<2>(ctx, i0, ni, P, runs, items, C, frags, cnorm, labels, rs, objpart, boxes, last_pass);
        case 3: return launch_split<3>(ctx, i0, ni, P, runs, items, C, frags, cnorm, labels, rs, objpart, boxes, last_pass);
        case 4: return launch_split<4>(ctx, i0, ni, P, runs, items, C, frags, cnorm, labels, rs, objpart, boxes, last_pass);
        default: return set_err(ctx, SUBKM_EINVAL, "split path: %d attribute steps", S);
    }
}

subkm_status wide_update(subkm_ctx *ctx, int r0, int nr, int i0, int ni, int w0, int nw, int u0,
                         int nu, const float *P, const DevRun *runs, const Item *items,
                         const int32_t *labels, float *C, RunState *rs, int32_t *cnt,
                         int32_t *order, int64_t olab_off, long long *gsum, double tol) {
    if (nr <= 0) return SUBKM_OK;
    ProfScope ps(ctx, PK_UPDATE);
    hipStream_t s = ctx->stream;
    const int nchunks = (int)ceil_div(ni, kChunkItems);
    if (ni > 0) {
        hipLaunchKernelGGL(k_wcount, dim3(nchunks), dim3(kAT), 0, s, runs, items, i0, ni, labels,
                           rs, cnt);
        SUBKM_LAUNCHED(ctx);
    }
    hipLaunchKernelGGL(k_wscan, dim3(nr), dim3(kAT), 0, s, runs, r0, rs, cnt);
    SUBKM_LAUNCHED(ctx);
    if (ni > 0) {
        hipLaunchKernelGGL(k_wscatter, dim3(nchunks), dim3(kAT), 0, s, runs, items, i0, ni, labels,
                           rs, cnt, order, olab_off);
        SUBKM_LAUNCHED(ctx);
    }
    if (nw > 0) {
        hipLaunchKernelGGL(k_wwalk, dim3(nw), dim3(kAT), 0, s, P, runs, items, w0, order, olab_off, C,
                           rs, cnt, gsum);
        SUBKM_LAUNCHED(ctx);
    }
    if (nu > 0) {
        hipLaunchKernelGGL(k_wfin, dim3(nu), dim3(kAT), 0, s, P, runs, items, u0, order, C, rs, cnt,
                           gsum, tol);
        SUBKM_LAUNCHED(ctx);
    }
    return SUBKM_OK;
}

}  // namespace subkm_lloyd
