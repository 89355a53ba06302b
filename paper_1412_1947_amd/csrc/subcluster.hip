// Equal sized subclustering (Sec. II, Algorithm 1 steps 2, 3 and 5), applied
// round after round to the points left over.
//
// One round is four launches with no host round trip (the threshold stays in
// device memory) and no inter-block synchronisation inside a kernel:
//
//   k_keys     binary64 key of every remaining point (its squared Euclidean or
//              its Manhattan distance to the landmark, attributes left to
//              right, no FMA) and a 4096-bin
//              histogram of a monotone 24-bit image v(key) of the key, merged
//              into 16 replicas so that no address sees many atomics, with
//              the counts of its 64-bin groups beside them;
//   k_cand     per block of 2048 positions: finds the bin a* holding the N-th
//              smallest key (group counts first, then the bins of that group),
//              counts the points surely selected (bin < a*) and compacts the
//              points of bin a* (candidates) into the block's own segment,
//              with a histogram of their low 12 bits;
//   k_sel2     (one block) finds the sub-bin, ranks the few candidates whose v
//              equals the boundary value exactly by (key, position), which
//              gives the threshold pair (key*, pos*), and turns the per-block
//              counts into output offsets;
//   k_scatter  stable compaction: a point is selected iff (key, pos) <=
//              (key*, pos*); selected rows go to P / perm in ascending index,
//              the others to the next remaining list, and every block folds
//              the attribute-wise minimum of the points it keeps into the
//              next landmark L_{t+1} (Algorithm 1 step 2 on the points left
//              over) with integer atomic minima on order-preserving bits,
//              and clears the level-1 histograms for the next round.  In
//              rounds where some point holding each attribute's minimum
//              surely stays (k_sel2 decides it from the largest key among
//              those holders), L_{t+1} = L_t and the early-load form reads
//              only the selected rows.
//
// Positions in the remaining list are in ascending original index, so the
// index tie-break of the selection is a tie-break on positions.
#include "internal.h"

#include <algorithm>
#include <cstring>

#pragma clang fp contract(off)

namespace {

constexpr int kT = 512;           // threads of the wide kernels
constexpr int kST = 1024;         // threads of the single-block kernels
constexpr int kBins = 4096;       // histogram bins per level
constexpr int kRep = 16;          // histogram replicas (spread the atomics)
constexpr int kGroups = kBins / 64;  // 64-bin groups of the level-1 bins
constexpr uint32_t kBS = 2048;    // positions per compaction block
constexpr int kRankCap = 2048;    // boundary candidates ranked in LDS
constexpr uint32_t kVMax = 0xFFFFFFu;
// remaining points from which the compaction reads only the selected rows in
// rounds whose landmark surely stays
constexpr uint32_t kSkipMin = 1u << 16;

struct SelState {
    uint32_t base;     // v-map offset of this round
    uint32_t astar, below1, cnt1;
    uint32_t bstar, below2, cnt2, need2;
    uint32_t thr_pos;
    uint32_t fallback;  // rounds that needed the slow exact path
    uint32_t ncand;     // length of the flat candidate list
    uint32_t vshift;    // low float bits the v-map drops this round
    uint32_t lchange;   // 0: no point holding an attribute minimum can be removed
    uint32_t sel_done;  // batched rounds: the threshold step of this pass is published
    double thr_key;
};

// Monotone non-decreasing map of a non-negative key to [0, 2^24): float32
// rounding (monotone), its bit pattern without the `sh` lowest bits, offset by
// `base`, clamped at both ends.  Any base and shift give an exact selection;
// they only decide how many keys share the boundary bins.
__device__ __forceinline__ uint32_t vmap(double key, uint32_t base, uint32_t sh) {
    uint32_t u = __float_as_uint((float)key) >> sh;
    uint32_t v = u > base ? u - base : 0u;
    return v > kVMax ? kVMax : v;
}

// The round's map.  Without a previous threshold: 4 bits dropped (the 2^24
// values span 32 binades) and the largest possible key in the top bin.
// Otherwise the threshold moves little from one round to the next, so the map
// is centred on the previous one with 2 bits dropped (8 binades, a quarter of
// them below it): a boundary bin then holds about a quarter of the keys it
// would hold under the bound-based map.
__device__ __forceinline__ void vmap_params(double bound, double prev_thr, bool have_prev,
                                            uint32_t *base, uint32_t *sh) {
    if (have_prev && prev_thr > 0.0) {
        const uint32_t c = __float_as_uint((float)prev_thr) >> 2;
        *sh = 2;
        *base = c > kVMax / 4 ? c - kVMax / 4 : 0u;
    } else {
        const uint32_t top = __float_as_uint((float)bound) >> 4;
        *sh = 4;
        *base = top > kVMax ? top - kVMax : 0u;
    }
}

__device__ __forceinline__ bool pair_le(double ka, uint32_t pa, double kb, uint32_t pb) {
    return ka < kb || (ka == kb && pa <= pb);
}

// Rows as float4 vectors (W = 4) or single floats (W = 1).
template <int W>
struct VecT;
template <>
struct VecT<1> {
    typedef float type;
};
template <>
struct VecT<4> {
    typedef float4 type;
};

__device__ __forceinline__ float vget(const float &v, int) { return v; }
__device__ __forceinline__ float vget(const float4 &v, int c) {
    return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w;
}

// Inclusive prefix sum over the 64 lanes of a wavefront in registers (DPP
// row shifts within each row of 16 lanes, then the row broadcasts of lanes
// 15 and 31), with no LDS round trip.  Every lane must be active.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// The same for 64-bit values (each step moves both halves, then adds with carry).
__device__ __forceinline__ unsigned long long wave_incl_scan64(unsigned long long x) {
#define SUBKM_SCAN64_STEP(ctrl, rmask)                                                              \
    {                                                                                              \
        const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, ctrl, rmask, 0xf, false); \
        const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), ctrl, rmask, 0xf, false); \
        x += ((unsigned long long)hi << 32) | lo;                                                  \
    }
    SUBKM_SCAN64_STEP(0x111, 0xf)
    SUBKM_SCAN64_STEP(0x112, 0xf)
    SUBKM_SCAN64_STEP(0x114, 0xf)
    SUBKM_SCAN64_STEP(0x118, 0xf)
    SUBKM_SCAN64_STEP(0x142, 0xa)
    SUBKM_SCAN64_STEP(0x143, 0xc)
#undef SUBKM_SCAN64_STEP
    return x;
}

// Exclusive scan of one value per thread over an NT-thread block.  Returns
// the prefix; *total receives the block sum.  `tmp` holds NT/64 words.
template <int NT>
__device__ uint32_t block_scan(uint32_t v, uint32_t *tmp, uint32_t *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t x = wave_incl_scan(v);
    if (lane == 63) tmp[wave] = x;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
    for (int w = 0; w < NT / 64; ++w) {
        uint32_t s = tmp[w];
        if (w < wave) wbase += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wbase + x - v;
}

// Sum the REP replicas of a kBins histogram (zeroing them for the next use
// when ZERO) and find the bin holding the need-th element (1-based).  Every
// thread of the kST-thread block returns the same (bin, below, count).
template <int REP, bool ZERO>
__device__ void merge_find_bin(uint32_t *hist, uint32_t need, uint32_t *sh, uint32_t *tmp,
                               uint32_t *bin, uint32_t *below, uint32_t *count) {
    constexpr int per = kBins / kST;
    if (threadIdx.x == 0) sh[0] = sh[1] = sh[2] = 0;
    uint32_t h[per], s = 0;
#pragma unroll
    for (int q = 0; q < per; ++q) {
        const int b = threadIdx.x * per + q;
        uint32_t a = 0;
#pragma unroll
        for (int r = 0; r < REP; ++r) {
            a += hist[r * kBins + b];
            if (ZERO) hist[r * kBins + b] = 0;
        }
        h[q] = a;
        s += a;
    }
    uint32_t tot;
    uint32_t cum = block_scan<kST>(s, tmp, &tot);
    if (cum < need && need <= cum + s) {
#pragma unroll
        for (int q = 0; q < per; ++q) {
            if (cum + h[q] >= need) {
                sh[0] = threadIdx.x * per + q;
                sh[1] = cum;
                sh[2] = h[q];
                break;
            }
            cum += h[q];
        }
    }
    __syncthreads();
    *bin = sh[0];
    *below = sh[1];
    *count = sh[2];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// The key of a point: M = 0 squared Euclidean, M = 1 Manhattan distance to the
// landmark (binary64, attributes left to right, no FMA).
template <int M>
__device__ __forceinline__ double key_term(double q) {
    return M ? fabs(q) : q * q;
}

// Add a block's histogram h to replica (block % kRep) of the level-1 bins and
// of their 64-bin group counts (those follow the bin replicas).  With kT a
// multiple of 64 and kBins of kT, each wave holds exactly one group per pass.
__device__ __forceinline__ void flush_hist(const uint32_t *h, uint32_t *hist1) {
    static_assert(kT % 64 == 0 && kBins % kT == 0, "a wave covers one group per pass");
    const uint32_t r = blockIdx.x % kRep;
    uint32_t *rep = hist1 + r * kBins;
    uint32_t *grp = hist1 + kRep * kBins + r * kGroups;
    for (int i = threadIdx.x; i < kBins; i += kT) {
        const uint32_t c = h[i];
        if (c) atomicAdd(&rep[i], c);
        uint32_t g = c;
        for (int o = 32; o > 0; o >>= 1) g += __shfl_xor(g, o, 64);
        if ((threadIdx.x & 63) == 0 && g) atomicAdd(&grp[i >> 6], g);
    }
}

template <int M>
__global__ __launch_bounds__(kT) void k_keys(const float *__restrict__ S, int d,
                                             const int32_t *__restrict__ rem, uint32_t nrem,
                                             const float *__restrict__ L,
                                             const uint32_t *__restrict__ Lcur, uint32_t *Lnext,
                                             const float *__restrict__ colmax,
                                             double *__restrict__ keys, uint32_t *hist1,
                                             SelState *st, float *landmarks_t, int vec4,
                                             int have_prev) {
    extern __shared__ float sL[];  // d floats
    __shared__ uint32_t h[kBins];
    __shared__ double s_term[kT];  // bound terms of the first kT attributes
    __shared__ uint32_t s_base, s_sh;
    for (int i = threadIdx.x; i < kBins; i += kT) h[i] = 0;
    for (int j = threadIdx.x; j < d; j += kT) {
        const float l = Lcur ? ordered_float(Lcur[j]) : L[j];
        sL[j] = l;
        if (j < kT) s_term[j] = key_term<M>((double)colmax[j] - (double)l);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // upper bound of any key of this round: sum_j term(max_j - L_j),
        // added left to right like the keys (the terms were formed in
        // parallel above)
        double b = 0.0;
        for (int j = 0; j < d; ++j) {
            const double t = j < kT ? s_term[j] : key_term<M>((double)colmax[j] - (double)sL[j]);
            b = b + t;
        }
        // (every block forms the same map; the previous round's threshold is
        // read before any block of this round can change it)
        uint32_t vb, vs;
        vmap_params(b, have_prev ? st->thr_key : 0.0, have_prev != 0, &vb, &vs);
        s_base = vb;
        s_sh = vs;
        if (blockIdx.x == 0) {
            st->base = vb;
            st->vshift = vs;
            st->ncand = 0;  // the candidate pass appends to it
        }
    }
    __syncthreads();
    if (blockIdx.x == 0)
        for (int j = threadIdx.x; j < d; j += kT) {
            if (landmarks_t) landmarks_t[j] = sL[j];
            if (Lnext) Lnext[j] = 0xFFFFFFFFu;  // the round's compaction folds the next landmark here
        }
    const uint32_t base = s_base, vsh = s_sh;
    for (uint32_t p = blockIdx.x * kT + threadIdx.x; p < nrem; p += gridDim.x * kT) {
        const float *row = S + (int64_t)rem[p] * d;
        double key = 0.0;
        if (vec4) {
            const float4 *r4 = (const float4 *)row;
            for (int j4 = 0; j4 < (d >> 2); ++j4) {
                float4 x = r4[j4];
                double q;
                q = (double)x.x - (double)sL[4 * j4 + 0]; key = key + key_term<M>(q);
                q = (double)x.y - (double)sL[4 * j4 + 1]; key = key + key_term<M>(q);
                q = (double)x.z - (double)sL[4 * j4 + 2]; key = key + key_term<M>(q);
                q = (double)x.w - (double)sL[4 * j4 + 3]; key = key + key_term<M>(q);
            }
        } else {
            for (int j = 0; j < d; ++j) {
                double q = (double)row[j] - (double)sL[j];
                key = key + key_term<M>(q);
            }
        }
        keys[p] = key;
        atomicAdd(&h[vmap(key, base, vsh) >> 12], 1u);
    }
    __syncthreads();
    flush_hist(h, hist1);
}

// The same keys for rows of a compile-time width D (float4 vectors when V4),
// PP points per thread at the grid stride.  The index and the whole row of
// every point of the thread are requested before the landmark and the map of
// the round are set up (those wait on their own loads and two barriers), so
// a thread makes two dependent memory round trips in all instead of two per
// point.  Keys and histograms are those of k_keys.
//
// Keys carried over: the compaction of the previous round wrote the key of
// every point that stayed, in the new order, to `keys`.  A key depends only on
// the row and the landmark, so when the landmark of this round equals the
// previous one bit for bit (reuse = 1; Lprev holds the previous landmark), or
// never moves (reuse = 2, fixed landmark), those keys are this round's and no
// row is read.  Removing a subcluster leaves the attribute-wise minimum
// unchanged whenever no removed point held a minimum, which is most rounds.
// Lsave (first round only) receives the landmark as ordered bits for the
// next round's comparison.
template <int M, int D, bool V4, int PP>
__global__ __launch_bounds__(kT) void k_keys_fast(const float *__restrict__ S,
                                                  const int32_t *__restrict__ rem, uint32_t nrem,
                                                  const float *__restrict__ L,
                                                  const uint32_t *__restrict__ Lcur,
                                                  uint32_t *Lnext, const float *__restrict__ colmax,
                                                  double *__restrict__ keys, uint32_t *hist1,
                                                  SelState *st, float *landmarks_t,
                                                  int have_prev, int reuse,
                                                  const uint32_t *__restrict__ Lprev,
                                                  uint32_t *__restrict__ Lsave,
                                                  unsigned long long *__restrict__ mk,
                                                  const unsigned long long *__restrict__ mk_prev) {
    constexpr int W = V4 ? 4 : 1;
    constexpr int NV = D / W;  // loads per row
    static_assert(D % W == 0 && D <= kT, "row width");
    typedef typename VecT<W>::type V;
    __shared__ float sL[D];
    __shared__ double s_term[D];
    __shared__ uint32_t h[kBins];
    __shared__ uint32_t s_base, s_sh;
    const uint32_t stride = gridDim.x * kT;
    const uint32_t p0 = blockIdx.x * kT + threadIdx.x;
    // the landmark test reads the same words in every thread (scalar loads):
    // every block takes the same branch
    bool same = reuse == 2;
    if (reuse == 1) {
        uint32_t diff = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) diff |= Lcur[j] ^ Lprev[j];
        same = diff == 0;
    }
    int32_t idx[PP];
    double kold[PP];
    if (same) {
#pragma unroll
        for (int u = 0; u < PP; ++u) {
            kold[u] = keys[min(p0 + u * stride, nrem - 1)];
            idx[u] = 0;
        }
    } else {
#pragma unroll
        for (int u = 0; u < PP; ++u) {
            const uint32_t p = min(p0 + u * stride, nrem - 1);
            idx[u] = rem ? rem[p] : (int32_t)p;
            kold[u] = 0.0;
        }
    }
    // unconditional loads (one pointer chosen for the whole grid, no branch)
    const int jl = threadIdx.x < D ? (int)threadIdx.x : D - 1;
    const uint32_t lraw = (Lcur ? Lcur : (const uint32_t *)L)[jl];
    const float cm = colmax[jl];
    const float lj = Lcur ? ordered_float(lraw) : __uint_as_float(lraw);
    const double prev = have_prev ? st->thr_key : 0.0;
    V x[PP][NV];
    if (!same) {
#pragma unroll
        for (int u = 0; u < PP; ++u)
#pragma unroll
            for (int q = 0; q < NV; ++q) x[u][q] = ((const V *)(S + (int64_t)idx[u] * D))[q];
    }

    for (int i = threadIdx.x; i < kBins; i += kT) h[i] = 0;
    if (threadIdx.x < D) {
        sL[threadIdx.x] = lj;
        s_term[threadIdx.x] = key_term<M>((double)cm - (double)lj);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // the key bound, added left to right like the keys
        double b = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) b = b + s_term[j];
        uint32_t vb, vs;
        vmap_params(b, prev, have_prev != 0, &vb, &vs);
        s_base = vb;
        s_sh = vs;
        if (blockIdx.x == 0) {
            st->base = vb;
            st->vshift = vs;
            st->ncand = 0;  // the candidate pass appends to it
        }
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x < D) {
        if (landmarks_t) landmarks_t[threadIdx.x] = sL[threadIdx.x];
        if (Lnext) Lnext[threadIdx.x] = 0xFFFFFFFFu;  // the round's compaction folds the next landmark here
        if (Lsave) Lsave[threadIdx.x] = ordered_bits(sL[threadIdx.x]);
        // same landmark, same keys: the holders' largest keys carry over
        if (mk && same) mk[threadIdx.x] = mk_prev[threadIdx.x];
    }
    const uint32_t base = s_base, vsh = s_sh;
#pragma unroll
    for (int u = 0; u < PP; ++u) {
        const uint32_t p = p0 + u * stride;
        double key = kold[u];
        if (!same) {
            key = 0.0;
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int c = 0; c < W; ++c) {
                    const double t = (double)vget(x[u][q], c) - (double)sL[q * W + c];
                    key = key + key_term<M>(t);
                }
        }
        if (p < nrem) {
            if (!same) keys[p] = key;
            atomicAdd(&h[vmap(key, base, vsh) >> 12], 1u);
            if (mk && !same) {
                // attributes in which this point holds the landmark (the
                // minimum): its key raises their holders' largest key
                uint32_t hold = 0;
#pragma unroll
                for (int q = 0; q < NV; ++q)
#pragma unroll
                    for (int c = 0; c < W; ++c)
                        hold |= (__float_as_uint(vget(x[u][q], c)) == __float_as_uint(sL[q * W + c])
                                     ? 1u : 0u) << (q * W + c);
                if (hold) {
                    const unsigned long long kb = (unsigned long long)__double_as_longlong(key);
                    for (int j = 0; j < D; ++j)
                        if ((hold >> j) & 1u) atomicMax(&mk[j], kb);
                }
            }
        }
    }
    __syncthreads();
    flush_hist(h, hist1);
}

typedef void (*KeysFastFn)(const float *, const int32_t *, uint32_t, const float *,
                           const uint32_t *, uint32_t *, const float *, double *, uint32_t *,
                           SelState *, float *, int, int, const uint32_t *, uint32_t *,
                           unsigned long long *, const unsigned long long *);

template <int M, int D, bool V4>
KeysFastFn keys_fast_pp(int pp) {
    return pp >= 4 ? k_keys_fast<M, D, V4, 4> : pp == 2 ? k_keys_fast<M, D, V4, 2>
                                                         : k_keys_fast<M, D, V4, 1>;
}

template <int M>
KeysFastFn keys_fast_m(int d, bool vec4, int pp) {
    switch (d) {
        case 1: return keys_fast_pp<M, 1, false>(pp);
        case 2: return keys_fast_pp<M, 2, false>(pp);
        case 4: return vec4 ? keys_fast_pp<M, 4, true>(pp) : nullptr;
        case 8: return vec4 ? keys_fast_pp<M, 8, true>(pp) : nullptr;
        case 16: return vec4 ? keys_fast_pp<M, 16, true>(pp) : nullptr;
        case 32: return vec4 ? keys_fast_pp<M, 32, true>(pp) : nullptr;
        default: return nullptr;
    }
}

// Points per thread of the early-load keys pass for nrem remaining points.
int keys_fast_pp_of(uint32_t nrem) { return nrem > (1u << 19) ? 4 : nrem > (1u << 18) ? 2 : 1; }

// The early-load keys pass for this metric, row width and alignment, or null.
KeysFastFn keys_fast_for(int metric, int d, bool vec4, int pp) {
    return metric ? keys_fast_m<1>(d, vec4, pp) : keys_fast_m<0>(d, vec4, pp);
}

// The level-1 bin a* holding the need-th smallest v (1-based) and the counts
// below and in it, from the kRep replicas written by the keys pass: first the
// 64-bin group from the group counts, then the bin inside that group (two
// reads of kRep x 64 words).  s_part: kT words of LDS.  Every thread of the
// kT-thread block returns the same values.
__device__ void find_bin1(const uint32_t *hist1, uint32_t need, uint32_t *s_part,
                          uint32_t *s_res, uint32_t *bin, uint32_t *below, uint32_t *count) {
    static_assert(kT == 8 * 64 && kRep == 16 && kGroups == 64, "two replicas per thread");
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_res[0] = s_res[1] = s_res[2] = 0;
    uint32_t at = 0, under = 0;
#pragma unroll
    for (int lev = 0; lev < 2; ++lev) {
        // lev 0: the group counts; lev 1: the 64 bins of group `at`
        const uint32_t *src = lev == 0 ? hist1 + kRep * kBins + lane : hist1 + at * 64 + lane;
        const uint32_t stride = lev == 0 ? kGroups : kBins;
        s_part[threadIdx.x] = src[w * stride] + src[(w + 8) * stride];
        __syncthreads();
        if (w == 0) {
            uint32_t c = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) c += s_part[q * 64 + lane];
            const uint32_t inc = wave_incl_scan(c);
            const uint32_t ex = under + inc - c;
            if (ex < need && need <= ex + c) {
                s_res[0] = lane;
                s_res[1] = ex;
                s_res[2] = c;
            }
        }
        __syncthreads();
        at = at * 64 + s_res[0];
        under = s_res[1];
    }
    *bin = at;
    *below = under;
    *count = s_res[2];
}

__global__ __launch_bounds__(kT) void k_cand(const double *__restrict__ keys, uint32_t nrem,
                                             uint32_t need, SelState *st,
                                             double *__restrict__ ckey,
                                             uint32_t *__restrict__ cpos,
                                             const uint32_t *hist1, uint32_t *hist2,
                                             uint32_t *__restrict__ blockcnt) {
    __shared__ uint32_t h[kBins];
    __shared__ double s_ck[kBS];
    __shared__ uint32_t s_cp[kBS];
    __shared__ uint32_t s_red[kT / 64], s_nc, s_base, s_res[3];
    const uint32_t base = st->base, vsh = st->vshift;
    const int lane = threadIdx.x & 63;
    uint32_t below = 0;
    const uint32_t p0 = blockIdx.x * kBS;
    constexpr int kPer = kBS / kT;
    double kb[kPer];  // all of the thread's keys in flight at once
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const uint32_t p = p0 + u * kT + threadIdx.x;
        kb[u] = keys[min(p, nrem - 1)];  // clamped, unconditional
    }
    // every block finds the boundary bin itself (h serves as scratch)
    uint32_t astar, below1, cnt1;
    find_bin1(hist1, need, h, s_res, &astar, &below1, &cnt1);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->astar = astar;
        st->below1 = below1;
        st->cnt1 = cnt1;
    }
    for (int i = threadIdx.x; i < kBins; i += kT) h[i] = 0;
    if (threadIdx.x == 0) s_nc = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const uint32_t p = p0 + u * kT + threadIdx.x;
        const bool in = p < nrem;
        const double k = kb[u];
        const uint32_t v = in ? vmap(k, base, vsh) : 0u;
        const uint32_t a = v >> 12;
        below += (in && a < astar) ? 1u : 0u;
        const bool c = in && a == astar;
        const uint64_t m = __ballot(c);
        if (m) {
            const uint32_t cnt = (uint32_t)__popcll(m);
            const uint32_t first = (uint32_t)__ffsll((unsigned long long)m) - 1;
            uint32_t slot0 = 0;
            if (lane == (int)first) slot0 = atomicAdd(&s_nc, cnt);
            slot0 = (uint32_t)__builtin_amdgcn_readlane((int)slot0, (int)first);
            if (c) {
                const uint32_t slot = slot0 + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
                s_ck[slot] = k;
                s_cp[slot] = p;
                atomicAdd(&h[v & 0xFFFu], 1u);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) below += __shfl_xor(below, o, 64);
    if (lane == 0) s_red[threadIdx.x >> 6] = below;
    __syncthreads();
    const uint32_t nc = s_nc;
    if (threadIdx.x == 0) {
        uint32_t sum = 0;
        for (int w = 0; w < kT / 64; ++w) sum += s_red[w];
        blockcnt[blockIdx.x] = sum;
        // the block's candidates go to one contiguous stretch of the list
        s_base = nc ? atomicAdd(&st->ncand, nc) : 0u;
    }
    __syncthreads();
    if (nc) {
        const uint32_t b0 = s_base;
        for (uint32_t i = threadIdx.x; i < nc; i += kT) {
            ckey[b0 + i] = s_ck[i];
            cpos[b0 + i] = s_cp[i];
        }
        // one histogram: only the candidates of one bin add to it
        for (int i = threadIdx.x; i < kBins; i += kT)
            if (h[i]) atomicAdd(&hist2[i], h[i]);
    }
}

// Exact selection of the need2-th smallest (key, pos) among the candidates
// whose v equals vstar, when there are too many to rank in LDS: a
// most-significant-digit radix select over the 96-bit pair, 8 bits a pass.
template <int NT>
__device__ void slow_select(const double *ckey, const uint32_t *cpos, uint32_t ncand,
                            uint32_t vstar, uint32_t base, uint32_t vsh, uint32_t need,
                            uint32_t *hist256, uint32_t *sh, double *thr_key, uint32_t *thr_pos) {
    uint64_t kpre = 0;
    uint32_t ppre = 0;
    for (int pass = 0; pass < 12; ++pass) {
        for (int i = threadIdx.x; i < 256; i += NT) hist256[i] = 0;
        __syncthreads();
        {
            for (uint32_t c = threadIdx.x; c < ncand; c += NT) {
                const double k = ckey[c];
                if (vmap(k, base, vsh) != vstar) continue;
                const uint64_t kb = (uint64_t)__double_as_longlong(k);
                const uint32_t p = cpos[c];
                bool match;
                uint32_t dig;
                if (pass < 8) {
                    const int hi = 64 - 8 * pass;  // bits above the current digit
                    match = pass == 0 || (kb >> hi) == (kpre >> hi);
                    dig = (uint32_t)(kb >> (56 - 8 * pass)) & 255u;
                } else {
                    const int q = pass - 8;
                    match = kb == kpre && (q == 0 || (p >> (32 - 8 * q)) == (ppre >> (32 - 8 * q)));
                    dig = (p >> (24 - 8 * q)) & 255u;
                }
                if (match) atomicAdd(&hist256[dig], 1u);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t cum = 0;
            for (int b = 0; b < 256; ++b) {
                if (cum + hist256[b] >= need) {
                    sh[0] = b;
                    sh[1] = cum;
                    break;
                }
                cum += hist256[b];
            }
        }
        __syncthreads();
        const uint32_t b = sh[0];
        need -= sh[1];
        if (pass < 8) kpre |= (uint64_t)b << (56 - 8 * pass);
        else ppre |= b << (24 - 8 * (pass - 8));
        __syncthreads();
    }
    *thr_key = __longlong_as_double((long long)kpre);
    *thr_pos = ppre;
}

constexpr uint32_t kSegCap = 4096;  // compaction blocks counted in LDS by k_sel2
constexpr int kBatch = 8;           // candidate loads in flight per thread in k_sel2

__global__ __launch_bounds__(kST) void k_sel2(uint32_t need, SelState *st,
                                              const double *__restrict__ ckey,
                                              const uint32_t *__restrict__ cpos, uint32_t nb,
                                              uint32_t *hist2, uint32_t *blockcnt,
                                              uint32_t *blockoff,
                                              const unsigned long long *__restrict__ mk, int d) {
    __shared__ uint32_t sh[4], tmp[kST / 64], s_n, s_lch;
    __shared__ double rk[kRankCap];
    __shared__ uint32_t rp[kRankCap];
    __shared__ uint32_t h256[256];
    __shared__ uint32_t csel[kSegCap];
    const uint32_t astar = st->astar, base = st->base, vsh = st->vshift;
    const uint32_t need1 = need - st->below1;
    const uint32_t ncand = st->ncand;
    const bool lds_counts = nb <= kSegCap;
    for (uint32_t i = threadIdx.x; i < kSegCap; i += kST) csel[i] = 0;
    uint32_t b, below2, cnt2;
    merge_find_bin<1, true>(hist2, need1, sh, tmp, &b, &below2, &cnt2);
    const uint32_t need2 = need1 - below2;
    const uint32_t vstar = (astar << 12) | b;
    // A candidate's bucket decides it unless it is the boundary bucket vstar
    // (the bucket map is monotone in the key): below, it is selected, and
    // joins its compaction block's count now; above, it stays.
    auto count_sel = [&](uint32_t pc) {
        if (lds_counts) atomicAdd(&csel[pc / kBS], 1u);
        else atomicAdd(&blockcnt[pc / kBS], 1u);
    };
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    for (uint32_t c0 = 0; c0 < ncand; c0 += kST * kBatch) {
        // the candidate list is thousands long: kBatch loads in flight per thread
        double kk[kBatch];
        uint32_t pp[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const uint32_t c = c0 + u * kST + threadIdx.x;
            const uint32_t cc = min(c, ncand - 1);  // clamped, unconditional
            kk[u] = ckey[cc];
            pp[u] = cpos[cc];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const uint32_t c = c0 + u * kST + threadIdx.x;
            if (c >= ncand) continue;
            const uint32_t v = vmap(kk[u], base, vsh);
            if (v < vstar) {
                count_sel(pp[u]);
            } else if (v == vstar) {
                const uint32_t q = atomicAdd(&s_n, 1u);
                if (q < (uint32_t)kRankCap) {
                    rk[q] = kk[u];
                    rp[q] = pp[u];
                }
            }
        }
    }
    __syncthreads();
    double thr_key;
    uint32_t thr_pos;
    if (cnt2 <= (uint32_t)kRankCap) {
        // exact rank of the few pairs in the boundary bucket
        for (uint32_t i = threadIdx.x; i < cnt2; i += kST) {
            const double ki = rk[i];
            const uint32_t pi = rp[i];
            uint32_t r = 0;
            for (uint32_t j = 0; j < cnt2; ++j) r += (rk[j] < ki || (rk[j] == ki && rp[j] < pi)) ? 1u : 0u;
            if (r == need2 - 1) sh[3] = i;
        }
        __syncthreads();
        thr_key = rk[sh[3]];
        thr_pos = rp[sh[3]];
        for (uint32_t i = threadIdx.x; i < cnt2; i += kST)
            if (pair_le(rk[i], rp[i], thr_key, thr_pos)) count_sel(rp[i]);
    } else {
        slow_select<kST>(ckey, cpos, ncand, vstar, base, vsh, need2, h256, sh, &thr_key, &thr_pos);
        if (threadIdx.x == 0) st->fallback += 1;
        for (uint32_t c = threadIdx.x; c < ncand; c += kST) {
            const double k = ckey[c];
            const uint32_t pc = cpos[c];
            if (vmap(k, base, vsh) == vstar && pair_le(k, pc, thr_key, thr_pos)) count_sel(pc);
        }
    }
    // The landmark can move only if every point holding some attribute's
    // minimum is removed, which needs that attribute's largest holder key to
    // be <= key* (an equal key is counted as removed: a conservative test)
    if (threadIdx.x == 0) s_lch = mk ? 0u : 1u;
    if (!lds_counts) __threadfence_block();
    __syncthreads();
    if (mk && (int)threadIdx.x < d &&
        mk[threadIdx.x] <= (unsigned long long)__double_as_longlong(thr_key))
        s_lch = 1u;
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < nb; c0 += kST) {
        const uint32_t sg = c0 + threadIdx.x;
        uint32_t v = 0;
        if (sg < nb) v = (lds_counts ? csel[sg] : 0u) + __hip_atomic_load(&blockcnt[sg], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t tot;
        const uint32_t pre = block_scan<kST>(v, tmp, &tot);
        if (sg < nb) blockoff[sg] = carry + pre;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        st->bstar = b;
        st->below2 = below2;
        st->cnt2 = cnt2;
        st->need2 = need2;
        st->thr_key = thr_key;
        st->thr_pos = thr_pos;
    }
    __syncthreads();
    if (threadIdx.x == 0) st->lchange = s_lch;
}


template <int W>
__device__ void scatter_rows(const float *__restrict__ S, int d, uint32_t cnt, const int32_t *s_src,
                             const int32_t *s_dst, int track_min, float *__restrict__ P,
                             int64_t off_t, uint32_t *s_cmin) {
    typedef typename VecT<W>::type V;
    constexpr int U = 8;
    const uint32_t dq = (uint32_t)d / W;
    const uint32_t total = cnt * dq;
    const uint32_t dr = kT / dq, dj = kT % dq;
    // a thread keeps its attribute group when kT is a multiple of dq
    const bool fixed = (kT % dq) == 0;
    uint32_t mymin[W];
#pragma unroll
    for (int c = 0; c < W; ++c) mymin[c] = 0xFFFFFFFFu;
    uint32_t r = threadIdx.x / dq, j = threadIdx.x % dq;
    const uint32_t j_fixed = j;
    for (uint32_t e = threadIdx.x; e < total; e += U * kT) {
        V v[U];
        int kind[U];  // 0: nothing to do, 1: copy to P row prow[u], 2: stays (minimum)
        int32_t prow[U];
        uint32_t jj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // every load is unconditional (past the block's rows the row
            // index is clamped to its last row, whose value is not used), so
            // the U loads are in flight together
            const uint32_t rc = min(r, cnt - 1);
            const int32_t dst = s_dst[rc];
            v[u] = ((const V *)(S + (int64_t)s_src[rc] * d))[j];
            const bool use = e + u * kT < total && dst != INT32_MIN;
            kind[u] = !use ? 0 : dst >= 0 ? 1 : 2;
            prow[u] = dst;
            jj[u] = j;
            r += dr;
            j += dj;
            if (j >= dq) {
                j -= dq;
                ++r;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (kind[u] == 1) {
                ((V *)(P + ((int64_t)off_t + prow[u]) * d))[jj[u]] = v[u];
            } else if (kind[u] == 2 && track_min) {
#pragma unroll
                for (int c = 0; c < W; ++c) {
                    const uint32_t o = ordered_bits(vget(v[u], c));
                    if (fixed) mymin[c] = min(mymin[c], o);
                    else atomicMin(&s_cmin[jj[u] * W + c], o);
                }
            }
        }
    }
    if (track_min && fixed && j_fixed < dq) {
#pragma unroll
        for (int c = 0; c < W; ++c)
            if (mymin[c] != 0xFFFFFFFFu) atomicMin(&s_cmin[j_fixed * W + c], mymin[c]);
    }
}

// ---------------------------------------------------------------------------
// Stable compaction of one block of kBS positions.  all_sel: every remaining
// point is selected (last round).  track_min: fold the attribute-wise
// minimum (ordered bits) of the points that stay into Lnext.
__global__ __launch_bounds__(kT) void k_scatter(const float *__restrict__ S, int d,
                                                const int32_t *__restrict__ rem,
                                                const double *__restrict__ keys, uint32_t nrem,
                                                uint32_t need, const SelState *__restrict__ st,
                                                const uint32_t *__restrict__ blockoff,
                                                int all_sel, int track_min, float *__restrict__ P,
                                                int32_t *__restrict__ perm, int64_t off_t,
                                                int32_t *__restrict__ rem_next,
                                                uint32_t *__restrict__ Lnext, int vec4,
                                                uint32_t *__restrict__ hclear) {
    __shared__ int32_t s_src[kBS];
    __shared__ int32_t s_dst[kBS];  // >= 0: P row; < 0: -(1 + slot) in rem_next
    __shared__ uint32_t tmp[kT / 64];
    __shared__ uint32_t s_min[kT];
    extern __shared__ uint32_t s_cmin[];  // d words (general-d path)
    constexpr int per = kBS / kT;
    const uint32_t p0 = blockIdx.x * kBS;
    const uint32_t cnt = min(kBS, nrem - p0);
    double thr_key = 0.0;
    uint32_t thr_pos = 0;
    if (!all_sel) {
        thr_key = st->thr_key;
        thr_pos = st->thr_pos;
    }
    // flags of this thread's `per` consecutive positions (unconditional
    // loads, clamped to the block's last position)
    double kq[per];
    int32_t iq[per];
#pragma unroll
    for (int q = 0; q < per; ++q) {
        const uint32_t pc = p0 + min(threadIdx.x * per + q, cnt - 1);
        kq[q] = all_sel ? 0.0 : keys[pc];
        iq[q] = rem ? rem[pc] : (int32_t)pc;
    }
    bool sel[per];
    uint32_t nsel = 0;
#pragma unroll
    for (int q = 0; q < per; ++q) {
        const uint32_t lp = threadIdx.x * per + q;
        const bool s = lp < cnt && (all_sel || pair_le(kq[q], p0 + lp, thr_key, thr_pos));
        sel[q] = s;
        nsel += s ? 1u : 0u;
    }
    uint32_t tot;
    const uint32_t pre = block_scan<kT>(nsel, tmp, &tot);
    const uint32_t sel_base = all_sel ? p0 : blockoff[blockIdx.x];
    const uint32_t stay_base = p0 - sel_base;
    uint32_t si = pre, ti = threadIdx.x * per - pre;
#pragma unroll
    for (int q = 0; q < per; ++q) {
        const uint32_t lp = threadIdx.x * per + q;
        if (lp < cnt) {
            const int32_t idx = iq[q];
            s_src[lp] = idx;
            // the guards only matter if the selection counts were inconsistent
            if (sel[q]) {
                const uint32_t row = sel_base + si++;
                const bool ok = row < need;
                s_dst[lp] = ok ? (int32_t)row : INT32_MIN;
                if (ok) perm[off_t + row] = idx;
            } else {
                const uint32_t slot = stay_base + ti++;
                const bool ok = slot < nrem - need;
                s_dst[lp] = ok ? -1 - (int32_t)slot : INT32_MIN;
                if (ok) rem_next[slot] = idx;
            }
        }
    }
    if (track_min)
        for (int j = threadIdx.x; j < d; j += kT) s_cmin[j] = 0xFFFFFFFFu;
    __syncthreads();
    // Rows: copy the selected ones, reduce the minimum of the others.  The
    // block's rows are walked as a flat array of W-float vectors (W = 4 when
    // d % 4 == 0), stepped by kT with no division in the loop; U vectors are
    // loaded before any is used so that several loads are in flight.
    if (track_min || tot > 0) {
        if (vec4) scatter_rows<4>(S, d, cnt, s_src, s_dst, track_min, P, off_t, s_cmin);
        else scatter_rows<1>(S, d, cnt, s_src, s_dst, track_min, P, off_t, s_cmin);
    }
    if (track_min) {
        // the next landmark: minimum over the blocks of the points that stay
        __syncthreads();
        for (int j = threadIdx.x; j < d; j += kT)
            if (s_cmin[j] != 0xFFFFFFFFu) atomicMin(&Lnext[j], s_cmin[j]);
    }
    // the level-1 replicas and group counts were last read by the candidate
    // pass: clear them for the next round, a slice per block
    {
        constexpr uint32_t words = kRep * (kBins + kGroups);
        const uint32_t zs = (words + gridDim.x - 1) / gridDim.x;
        const uint32_t z0 = blockIdx.x * zs, z1 = min(words, z0 + zs);
        for (uint32_t i = z0 + threadIdx.x; i < z1; i += kT) hclear[i] = 0;
    }
}

// The same compaction for rows of d = W * DQ attributes with DQ dividing kT
// (a thread keeps one attribute group j for all its vectors).  The rows a
// block touches are its own span of positions whatever the selection decides,
// so the row index of every vector is read straight from the remaining list
// and every row is requested before the keys are compared and scanned; the
// selection then only decides where each row goes.  Every load address is
// clamped into the block's span, so the loads are unconditional and go out
// together: two dependent memory round trips per block instead of one per
// key, index and row batch.  Results are those of k_scatter.
template <int W, int DQ>
__global__ __launch_bounds__(kT, W * DQ <= 16 ? 4 : 1) void k_scatter_fast(
    const float *__restrict__ S, const int32_t *__restrict__ rem,
    const double *__restrict__ keys, uint32_t nrem, uint32_t need,
    const SelState *__restrict__ st, const uint32_t *__restrict__ blockoff, int all_sel,
    int track_min, float *__restrict__ P, int32_t *__restrict__ perm, int64_t off_t,
    int32_t *__restrict__ rem_next, uint32_t *__restrict__ Lnext,
    double *__restrict__ keys_next, uint32_t *__restrict__ hclear, int lm_skip,
    const uint32_t *__restrict__ Lcur, const float *__restrict__ L,
    unsigned long long *__restrict__ mk_clear) {
    typedef typename VecT<W>::type V;
    constexpr int D = W * DQ;
    constexpr int per = kBS / kT;   // positions per thread in the selection
    constexpr int RS = kT / DQ;     // rows per sweep of the block
    constexpr int NV = kBS / RS;    // row vectors per thread
    static_assert(kT % DQ == 0 && kBS % RS == 0, "attribute groups must tile the block");
    __shared__ int32_t s_dst[kBS];  // >= 0: P row; < 0: -(1 + slot) in rem_next
    __shared__ uint32_t tmp[kT / 64];
    __shared__ uint32_t s_cmin[D];
    const uint32_t p0 = blockIdx.x * kBS;
    const uint32_t cnt = min(kBS, nrem - p0);
    const uint32_t last = p0 + cnt - 1;
    const int j = threadIdx.x % DQ;
    const uint32_t r0 = threadIdx.x / DQ;
    int32_t ridx[NV];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        const uint32_t p = min(p0 + r0 + u * RS, last);
        ridx[u] = rem ? rem[p] : (int32_t)p;
    }
    double kq[per];
    int32_t iq[per];
#pragma unroll
    for (int q = 0; q < per; ++q) {
        const uint32_t p = min(p0 + threadIdx.x * per + q, last);
        kq[q] = all_sel ? 0.0 : keys[p];
        iq[q] = rem ? rem[p] : (int32_t)p;
    }
    double thr_key = 0.0;
    uint32_t thr_pos = 0, sel_base = p0, lch = 1;
    if (!all_sel) {
        thr_key = st->thr_key;
        thr_pos = st->thr_pos;
        sel_base = blockoff[blockIdx.x];
        lch = st->lchange;
    }
    // Rows are needed for the selected points, and for the others only when
    // the next landmark has to be folded from them.  When the landmark
    // surely stays (or is fixed), only selected rows are read, after the
    // selection; otherwise every row is requested now (one uniform branch).
    const bool full = !(lm_skip && !all_sel && (!track_min || lch == 0));
    V v[NV];
    if (full) {
#pragma unroll
        for (int u = 0; u < NV; ++u) v[u] = ((const V *)(S + (int64_t)ridx[u] * D))[j];
    }

    bool sel[per];
    uint32_t nsel = 0;
#pragma unroll
    for (int q = 0; q < per; ++q) {
        const uint32_t lp = threadIdx.x * per + q;
        sel[q] = lp < cnt && (all_sel || pair_le(kq[q], p0 + lp, thr_key, thr_pos));
        nsel += sel[q] ? 1u : 0u;
    }
    uint32_t tot;
    const uint32_t pre = block_scan<kT>(nsel, tmp, &tot);
    const uint32_t stay_base = p0 - sel_base;
    uint32_t si = pre, ti = threadIdx.x * per - pre;
#pragma unroll
    for (int q = 0; q < per; ++q) {
        const uint32_t lp = threadIdx.x * per + q;
        if (lp < cnt) {
            // the guards only matter if the selection counts were inconsistent
            if (sel[q]) {
                const uint32_t row = sel_base + si++;
                const bool ok = row < need;
                s_dst[lp] = ok ? (int32_t)row : INT32_MIN;
                if (ok) perm[off_t + row] = iq[q];
            } else {
                const uint32_t slot = stay_base + ti++;
                const bool ok = slot < nrem - need;
                s_dst[lp] = ok ? -1 - (int32_t)slot : INT32_MIN;
                if (ok) {
                    rem_next[slot] = iq[q];
                    // the next round's keys pass may take it as is
                    if (keys_next) keys_next[slot] = kq[q];
                }
            }
        }
    }
    if (track_min && threadIdx.x < D) s_cmin[threadIdx.x] = 0xFFFFFFFFu;
    __syncthreads();
    if (!full) {
        // every thread loads; a row that is not selected reads row 0 instead
        // (one line for the whole grid), so the loads go out together
#pragma unroll
        for (int u = 0; u < NV; ++u) {
            const uint32_t rc = min(r0 + u * RS, cnt - 1);
            const int32_t row = s_dst[rc] >= 0 ? ridx[u] : 0;
            v[u] = ((const V *)(S + (int64_t)row * D))[j];
        }
    }
    const bool fold = track_min && full;
    uint32_t mymin[W];
#pragma unroll
    for (int c = 0; c < W; ++c) mymin[c] = 0xFFFFFFFFu;
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        const uint32_t r = r0 + u * RS;
        if (r < cnt) {
            const int32_t dst = s_dst[r];
            if (dst >= 0) {
                ((V *)(P + (off_t + dst) * D))[j] = v[u];
            } else if (fold && dst != INT32_MIN) {
#pragma unroll
                for (int c = 0; c < W; ++c) mymin[c] = min(mymin[c], ordered_bits(vget(v[u], c)));
            }
        }
    }
    if (fold) {
#pragma unroll
        for (int c = 0; c < W; ++c)
            if (mymin[c] != 0xFFFFFFFFu) atomicMin(&s_cmin[j * W + c], mymin[c]);
        // the next landmark: minimum over the blocks of the points that stay
        __syncthreads();
        if (threadIdx.x < D && s_cmin[threadIdx.x] != 0xFFFFFFFFu)
            atomicMin(&Lnext[threadIdx.x], s_cmin[threadIdx.x]);
    } else if (track_min && blockIdx.x == 0 && threadIdx.x < D) {
        // the landmark stays (every block takes this branch)
        Lnext[threadIdx.x] = Lcur ? Lcur[threadIdx.x] : ordered_bits(L[threadIdx.x]);
    }
    // the next round's holder keys start from zero
    if (mk_clear && blockIdx.x == 0 && threadIdx.x < D) mk_clear[threadIdx.x] = 0ull;
    // the level-1 replicas and group counts were last read by the candidate
    // pass: clear them for the next round, a slice per block
    {
        constexpr uint32_t words = kRep * (kBins + kGroups);
        const uint32_t zs = (words + gridDim.x - 1) / gridDim.x;
        const uint32_t z0 = blockIdx.x * zs, z1 = min(words, z0 + zs);
        for (uint32_t i = z0 + threadIdx.x; i < z1; i += kT) hclear[i] = 0;
    }
}

typedef void (*ScatterFastFn)(const float *, const int32_t *, const double *, uint32_t, uint32_t,
                              const SelState *, const uint32_t *, int, int, float *, int32_t *,
                              int64_t, int32_t *, uint32_t *, double *, uint32_t *, int,
                              const uint32_t *, const float *, unsigned long long *);

// The early-load compaction for this row width and alignment, or null.
ScatterFastFn scatter_fast_for(int d, bool vec4) {
    if (vec4) {
        switch (d) {
            case 4: return k_scatter_fast<4, 1>;
            case 8: return k_scatter_fast<4, 2>;
            case 16: return k_scatter_fast<4, 4>;
            case 32: return k_scatter_fast<4, 8>;
            default: return nullptr;
        }
    }
    switch (d) {
        case 1: return k_scatter_fast<1, 1>;
        case 2: return k_scatter_fast<1, 2>;
        case 4: return k_scatter_fast<1, 4>;
        case 8: return k_scatter_fast<1, 8>;
        default: return nullptr;
    }
}

__global__ void k_iota(int32_t *a, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = (int32_t)i;
}

__global__ void k_fill_u32(uint32_t *a, uint32_t n, uint32_t v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_bits_to_f32(float *dst, const uint32_t *src, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = ordered_float(src[i]);
}

__global__ void k_copy_f32(float *dst, const float *src, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void k_offsets(int64_t *off, int64_t T, int64_t N, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= T) off[t] = t < T ? t * N : n;
}

// ---------------------------------------------------------------------------
// Batches of rounds that share a landmark.
//
// Removing a subcluster leaves the landmark (the attribute-wise minimum of
// the remaining points) unchanged while, for every attribute, some point
// holding its minimum stays.  While the landmark stays, so do the keys, and
// the subclusters of rounds t, t+1, ..., t+q-1 are the consecutive N-blocks
// of one (key, position) order of the points remaining at round t.  The
// keys pass records, per attribute, the largest key among the points that
// hold the minimum (mk); every point with a smaller key ranks below that
// holder, so with c = #{keys < min_j mk_j} the landmark surely stays for
// rounds t+1 .. t + floor(c / N).  One batch therefore selects the ranks N,
// 2N, ..., qN at once (q <= kQMax, q - 1 <= floor(c / N), and the last round
// always left to a slot of its own), sorts the points into q subclusters
// and the rest in one compaction, and the rounds t+1 .. t+q-1 have nothing
// left to do.  With a fixed landmark every batch takes the largest q.
//
// The launch sequence stays static (it is captured once into a HIP graph):
// every round t keeps its three launches (keys pass, candidate pass, and the
// compaction whose block 0 first runs the threshold step), and act[t] says whether round t
// starts a batch (the number of batches before it, which also selects the
// ping-pong buffers) or lies inside an earlier one (kNoRound: every block
// returns at once).  A batch at round t writes act[t + q]; nothing else
// writes act during the sequence, so no launch reads a word another one of
// the same launch writes.
constexpr int kQMax = 9;                   // subclusters one batch emits at most
constexpr uint32_t kNoRound = 0xFFFFFFFFu;  // act[t]: round t lies inside a batch
constexpr uint32_t kCselCap = 8192;        // (class, block) counts the threshold step keeps in LDS

struct BatchPlan {
    uint32_t q;                 // subclusters of the active batch
    uint32_t lchange;           // 0: the landmark surely stays after the batch
    uint32_t bin[kQMax];        // level-1 bin of rank (i + 1) N
    uint32_t below[kQMax];      // points in bins below bin[i]
    uint32_t cnt[kQMax];        // points in bin[i]
    uint32_t thr_pos[kQMax];    // threshold of group i: (thr_key[i], thr_pos[i])
    double thr_key[kQMax];
};

// Buffers of the batched sequence (kernel arguments by value).
struct RoundBufs {
    const float *S;
    float *P;
    int32_t *perm;
    float *landmarks;            // nullable, T x d
    int32_t *rem[2];             // remaining positions -> index, by batch parity
    double *keys[2];             // keys of the remaining points, by batch parity
    uint32_t *Lb;                // 3 x d landmarks as ordered bits (batch count mod 3)
    unsigned long long *mk;      // 2 x d largest holder keys (nullptr: fixed landmark)
    const float *L0;             // first landmark
    const float *colmax;
    SelState *st;
    BatchPlan *bp;
    uint32_t *act;               // T + 1 words
    uint32_t *hist1;             // level-1 replicas and group counts (the keys pass)
    uint32_t *hist2;             // kQMax level-2 histograms
    uint32_t *blockcnt;          // (kQMax + 1) x nbs
    uint32_t *blockoff;          // (kQMax + 1) x nbs
    double *ckey;
    uint32_t *cpos;
    uint32_t nbs;                // stride of the per-class block arrays
    int32_t d;
    int *err;                    // sticky device flag: a bounded wait gave up
};

// The keys pass of a batch (k_keys_fast with the buffers of batch act[t]).
template <int M, int D, bool V4, int PP>
__global__ __launch_bounds__(kT) void k_keys_b(RoundBufs B, uint32_t t, uint32_t nrem, int fixed) {
    constexpr int W = V4 ? 4 : 1;
    constexpr int NV = D / W;
    static_assert(D % W == 0 && D <= kT, "row width");
    typedef typename VecT<W>::type V;
    const uint32_t a = B.act[t];
    if (a == kNoRound) return;
    __shared__ float sL[D];
    __shared__ double s_term[D];
    __shared__ uint32_t h[kBins];
    __shared__ uint32_t s_base, s_sh;
    const int32_t *rem = t == 0 ? nullptr : B.rem[a & 1];
    double *keys = B.keys[a & 1];
    const uint32_t *Lcur = (t == 0 || fixed) ? nullptr : B.Lb + (a % 3) * D;
    uint32_t *Lnext = fixed ? nullptr : B.Lb + ((a + 1) % 3) * D;
    const uint32_t *Lprev = (t > 0 && !fixed) ? B.Lb + ((a + 2) % 3) * D : nullptr;
    uint32_t *Lsave = (t == 0 && !fixed) ? B.Lb + (a % 3) * D : nullptr;
    unsigned long long *mk = B.mk ? B.mk + (a & 1) * D : nullptr;
    const unsigned long long *mk_prev = B.mk ? B.mk + ((a + 1) & 1) * D : nullptr;
    const int reuse = t == 0 ? 0 : fixed ? 2 : 1;
    const uint32_t stride = gridDim.x * kT;
    const uint32_t p0 = blockIdx.x * kT + threadIdx.x;
    bool same = reuse == 2;
    if (reuse == 1) {
        uint32_t diff = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) diff |= Lcur[j] ^ Lprev[j];
        same = diff == 0;
    }
    int32_t idx[PP];
    double kold[PP];
    if (same) {
#pragma unroll
        for (int u = 0; u < PP; ++u) {
            kold[u] = keys[min(p0 + u * stride, nrem - 1)];
            idx[u] = 0;
        }
    } else {
#pragma unroll
        for (int u = 0; u < PP; ++u) {
            const uint32_t p = min(p0 + u * stride, nrem - 1);
            idx[u] = rem ? rem[p] : (int32_t)p;
            kold[u] = 0.0;
        }
    }
    const int jl = threadIdx.x < D ? (int)threadIdx.x : D - 1;
    const uint32_t lraw = (Lcur ? Lcur : (const uint32_t *)B.L0)[jl];
    const float cm = B.colmax[jl];
    const float lj = Lcur ? ordered_float(lraw) : __uint_as_float(lraw);
    const double prev = t > 0 ? B.st->thr_key : 0.0;
    V x[PP][NV];
    if (!same) {
#pragma unroll
        for (int u = 0; u < PP; ++u)
#pragma unroll
            for (int q = 0; q < NV; ++q) x[u][q] = ((const V *)(B.S + (int64_t)idx[u] * D))[q];
    }
    for (int i = threadIdx.x; i < kBins; i += kT) h[i] = 0;
    if (threadIdx.x < D) {
        sL[threadIdx.x] = lj;
        s_term[threadIdx.x] = key_term<M>((double)cm - (double)lj);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) b = b + s_term[j];
        uint32_t vb, vs;
        vmap_params(b, prev, t > 0, &vb, &vs);
        s_base = vb;
        s_sh = vs;
        if (blockIdx.x == 0) {
            B.st->base = vb;
            B.st->vshift = vs;
            B.st->ncand = 0;
        }
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x < D) {
        if (B.landmarks) B.landmarks[(int64_t)t * D + threadIdx.x] = sL[threadIdx.x];
        if (Lnext) Lnext[threadIdx.x] = 0xFFFFFFFFu;
        if (Lsave) Lsave[threadIdx.x] = ordered_bits(sL[threadIdx.x]);
        if (mk && same) mk[threadIdx.x] = mk_prev[threadIdx.x];
    }
    const uint32_t base = s_base, vsh = s_sh;
#pragma unroll
    for (int u = 0; u < PP; ++u) {
        const uint32_t p = p0 + u * stride;
        double key = kold[u];
        if (!same) {
            key = 0.0;
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int c = 0; c < W; ++c) {
                    const double dlt = (double)vget(x[u][q], c) - (double)sL[q * W + c];
                    key = key + key_term<M>(dlt);
                }
        }
        if (p < nrem) {
            if (!same) keys[p] = key;
            atomicAdd(&h[vmap(key, base, vsh) >> 12], 1u);
            if (mk && !same) {
                uint32_t hold = 0;
#pragma unroll
                for (int q = 0; q < NV; ++q)
#pragma unroll
                    for (int c = 0; c < W; ++c)
                        hold |= (__float_as_uint(vget(x[u][q], c)) == __float_as_uint(sL[q * W + c])
                                     ? 1u : 0u) << (q * W + c);
                if (hold) {
                    const unsigned long long kb = (unsigned long long)__double_as_longlong(key);
                    for (int j = 0; j < D; ++j)
                        if ((hold >> j) & 1u) atomicMax(&mk[j], kb);
                }
            }
        }
    }
    __syncthreads();
    flush_hist(h, B.hist1);
}

typedef void (*KeysBFn)(RoundBufs, uint32_t, uint32_t, int);

template <int M, int D, bool V4>
KeysBFn keys_b_pp(int pp) {
    return pp >= 4 ? k_keys_b<M, D, V4, 4> : pp == 2 ? k_keys_b<M, D, V4, 2> : k_keys_b<M, D, V4, 1>;
}

template <int M>
KeysBFn keys_b_m(int d, bool vec4, int pp) {
    switch (d) {
        case 1: return keys_b_pp<M, 1, false>(pp);
        case 2: return keys_b_pp<M, 2, false>(pp);
        case 4: return vec4 ? keys_b_pp<M, 4, true>(pp) : nullptr;
        case 8: return vec4 ? keys_b_pp<M, 8, true>(pp) : nullptr;
        case 16: return vec4 ? keys_b_pp<M, 16, true>(pp) : nullptr;
        case 32: return vec4 ? keys_b_pp<M, 32, true>(pp) : nullptr;
        default: return nullptr;
    }
}

KeysBFn keys_b_for(int metric, int d, bool vec4, int pp) {
    return metric ? keys_b_m<1>(d, vec4, pp) : keys_b_m<0>(d, vec4, pp);
}

// Plan of a batch, computed by every block of k_candm alike from the
// level-1 histogram: the number of subclusters q, and for every target rank
// (i + 1) N the level-1 bin holding it with the counts below and in it.
// The group counts (64 bins a group) first; then one wave per target (and
// one for the holder key) finds its group with a ballot, reads that group's
// 64 bins and finds its bin with a scan and a ballot.
struct PlanLds {
    uint32_t part[kT];
    uint32_t gpre[kGroups + 1];      // exclusive prefix of the group totals
    uint32_t tbin[kQMax], tbelow[kQMax], tcnt[kQMax];
    uint32_t hkbelow;                // points in bins below the holder key's bin
    unsigned long long hk;           // smallest of the largest holder keys
    uint32_t q;
};

__device__ void batch_plan(const RoundBufs &B, uint32_t a, uint32_t t, uint32_t T, uint32_t N,
                           uint32_t base, uint32_t vsh, PlanLds &Lp) {
    static_assert(kT == 8 * 64 && kRep == 16 && kGroups == 64, "two replicas per thread");
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t *grp = B.hist1 + kRep * kBins;
    Lp.part[threadIdx.x] = grp[w * kGroups + lane] + grp[(w + 8) * kGroups + lane];
    if (threadIdx.x == 0) {
        unsigned long long hk = ~0ull;
        if (B.mk) {
            const unsigned long long *mk = B.mk + (a & 1) * B.d;
            for (int j = 0; j < B.d; ++j) hk = min(hk, mk[j]);
        }
        Lp.hk = hk;
        Lp.hkbelow = 0;
    }
    __syncthreads();
    if (w == 0) {
        uint32_t c = 0;
#pragma unroll
        for (int r = 0; r < 8; ++r) c += Lp.part[r * 64 + lane];
        const uint32_t inc = wave_incl_scan(c);
        Lp.gpre[lane] = inc - c;
        if (lane == 63) Lp.gpre[64] = inc;
    }
    __syncthreads();
    const uint32_t qcap = min((uint32_t)kQMax, T - 1 - t);
    // item i < qcap: target rank (i + 1) N; item kQMax: the holder key
    for (uint32_t i = w; i <= (uint32_t)kQMax; i += kT / 64) {
        const bool target = i < qcap;
        const bool holder = i == (uint32_t)kQMax && B.mk != nullptr;
        if (!target && !holder) continue;
        uint32_t g, hb = 0;
        const uint32_t rank = target ? (i + 1) * N : 0u;
        if (target) {
            const uint64_t m = __ballot(Lp.gpre[lane] < rank && rank <= Lp.gpre[lane + 1]);
            g = m ? (uint32_t)(__ffsll((unsigned long long)m) - 1) : 0u;
        } else {
            hb = vmap(__longlong_as_double((long long)Lp.hk), base, vsh) >> 12;
            g = hb >> 6;
        }
        uint32_t c = 0;
#pragma unroll
        for (int r = 0; r < kRep; ++r) c += B.hist1[r * kBins + g * 64 + lane];
        const uint32_t inc = wave_incl_scan(c);
        const uint32_t lo = Lp.gpre[g] + inc - c;  // points below bin g * 64 + lane
        if (target) {
            const uint64_t m = __ballot(lo < rank && rank <= lo + c);
            const int b = m ? __ffsll((unsigned long long)m) - 1 : 0;
            if (lane == b) {
                Lp.tbin[i] = g * 64 + b;
                Lp.tbelow[i] = lo;
                Lp.tcnt[i] = c;
            }
        } else if (lane == (int)(hb & 63)) {
            Lp.hkbelow = lo;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t q = qcap;
        // every key in a bin below the holder key's bin is below it
        if (B.mk) q = min(q, 1 + Lp.hkbelow / N);
        Lp.q = max(q, 1u);
    }
    __syncthreads();
}

// Candidate pass of a batch: the plan, then per block of kBS positions the
// points surely in each class (bin strictly between the boundary bins) and
// the candidates (a boundary bin) with their level-2 histograms, one per
// distinct boundary bin (the slot of its first target).
__global__ __launch_bounds__(kT) void k_candm(RoundBufs B, uint32_t t, uint32_t T, uint32_t nrem,
                                              uint32_t N) {
    const uint32_t a = B.act[t];
    if (a == kNoRound) return;
    __shared__ PlanLds Lp;
    __shared__ double s_ck[kBS];
    __shared__ uint32_t s_cp[kBS];
    __shared__ uint32_t s_cc[kQMax + 1];
    __shared__ uint32_t s_nc, s_base;
    const double *keys = B.keys[a & 1];
    const uint32_t base = B.st->base, vsh = B.st->vshift;
    const int lane = threadIdx.x & 63;
    const uint32_t p0 = blockIdx.x * kBS;
    constexpr int kPer = kBS / kT;
    double kb[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const uint32_t p = p0 + u * kT + threadIdx.x;
        kb[u] = keys[min(p, nrem - 1)];  // clamped, unconditional
    }
    if (threadIdx.x <= (uint32_t)kQMax) s_cc[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_nc = 0;
    batch_plan(B, a, t, T, N, base, vsh, Lp);
    const uint32_t q = Lp.q;
    if (blockIdx.x == 0 && threadIdx.x < q) {
        B.bp->bin[threadIdx.x] = Lp.tbin[threadIdx.x];
        B.bp->below[threadIdx.x] = Lp.tbelow[threadIdx.x];
        B.bp->cnt[threadIdx.x] = Lp.tcnt[threadIdx.x];
        if (threadIdx.x == 0) {
            B.bp->q = q;
            B.st->sel_done = 0;  // the compaction launch publishes this pass's thresholds
        }
    }
    // the targets' level-1 bins in registers (padding above every bin)
    uint32_t tb[kQMax];
#pragma unroll
    for (int i = 0; i < kQMax; ++i) tb[i] = (uint32_t)i < q ? Lp.tbin[i] : 0xFFFFFFFFu;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const uint32_t p = p0 + u * kT + threadIdx.x;
        const bool in = p < nrem;
        const uint32_t v = in ? vmap(kb[u], base, vsh) : 0u;
        const uint32_t b = v >> 12;
        uint32_t lo = 0, hi = 0;
#pragma unroll
        for (int i = 0; i < kQMax; ++i) {
            lo += tb[i] < b ? 1u : 0u;
            hi += tb[i] <= b ? 1u : 0u;
        }
        const bool sure = in && lo == hi;
        // sure points: one ballot per class present in the wave
        uint64_t rest = __ballot(sure);
        while (rest) {
            const int l0 = __ffsll((unsigned long long)rest) - 1;
            const uint32_t c0 = (uint32_t)__builtin_amdgcn_readlane((int)lo, l0);
            const uint64_t m = __ballot(sure && lo == c0);
            if (lane == l0) atomicAdd(&s_cc[c0], (uint32_t)__popcll(m));
            rest &= ~m;
        }
        const bool c = in && lo != hi;
        const uint64_t m = __ballot(c);
        if (m) {
            const uint32_t cnt = (uint32_t)__popcll(m);
            const uint32_t first = (uint32_t)__ffsll((unsigned long long)m) - 1;
            uint32_t slot0 = 0;
            if (lane == (int)first) slot0 = atomicAdd(&s_nc, cnt);
            slot0 = (uint32_t)__builtin_amdgcn_readlane((int)slot0, (int)first);
            if (c) {
                const uint32_t slot = slot0 + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
                s_ck[slot] = kb[u];
                s_cp[slot] = p;
                atomicAdd(&B.hist2[lo * kBins + (v & 0xFFFu)], 1u);
            }
        }
    }
    __syncthreads();
    const uint32_t nc = s_nc;
    if (threadIdx.x <= q) B.blockcnt[threadIdx.x * B.nbs + blockIdx.x] = s_cc[threadIdx.x];
    if (threadIdx.x == 0) s_base = nc ? atomicAdd(&B.st->ncand, nc) : 0u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nc; i += kT) {
        B.ckey[s_base + i] = s_ck[i];
        B.cpos[s_base + i] = s_cp[i];
    }
}

// Thresholds of a batch (one block: block 0 of the batch's compaction launch,
// the other blocks of which wait for it).  (1) For every distinct boundary bin,
// one wave scans its level-2 histogram (and clears it) and gives every target
// in it the level-2 bin of its rank.  (2) One pass over the candidate list:
// a candidate whose level-2 value differs from every target's is below or
// above each threshold by that value alone, so its class is known and it
// joins its compaction block's count at once; the others (the few sharing a
// target's level-2 bin) are gathered into that target's segment of LDS.
// (3) Exact ranks by (key, position) inside every segment give the
// thresholds, then the segment members get their classes.  A target whose
// level-2 bin holds too many candidates for LDS takes a radix select over
// the list, and then one more pass classifies the members of such bins.
// (4) Per class, one wave turns the block counts into offsets.  Then:
// whether the landmark may move after the batch, the round of the next
// batch, the landmarks of the rounds inside this one.
struct Sel2Lds {
    uint32_t sh[4], s_lch, s_anyslow;
    double rk[kRankCap];
    uint32_t rp[kRankCap];
    uint32_t h256[256];
    uint32_t csel[kCselCap];
    double s_tk[kQMax];
    uint32_t s_tp[kQMax], s_bin[kQMax], s_below[kQMax];
    uint32_t s_vstar[kQMax], s_need2[kQMax], s_cnt2[kQMax], s_seg[kQMax], s_fill[kQMax];
    uint32_t s_fast[kQMax];
};

template <int NT>
__device__ void sel2m_body(const RoundBufs &B, uint32_t t, uint32_t N, uint32_t nb, int fixed,
                           uint32_t a, Sel2Lds &S2) {
    uint32_t *sh = S2.sh;
    uint32_t &s_lch = S2.s_lch, &s_anyslow = S2.s_anyslow;
    double *rk = S2.rk;
    uint32_t *rp = S2.rp, *h256 = S2.h256, *csel = S2.csel;
    double *s_tk = S2.s_tk;
    uint32_t *s_tp = S2.s_tp, *s_bin = S2.s_bin, *s_below = S2.s_below, *s_vstar = S2.s_vstar;
    uint32_t *s_need2 = S2.s_need2, *s_cnt2 = S2.s_cnt2, *s_seg = S2.s_seg, *s_fill = S2.s_fill;
    uint32_t *s_fast = S2.s_fast;
    const BatchPlan *bp = B.bp;
    const uint32_t q = bp->q;
    const uint32_t base = B.st->base, vsh = B.st->vshift;
    const uint32_t ncand = B.st->ncand;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool lds_counts = (q + 1) * nb <= kCselCap;
    for (uint32_t i = threadIdx.x; i < kCselCap; i += NT) csel[i] = 0;
    if (threadIdx.x < q) {
        s_bin[threadIdx.x] = bp->bin[threadIdx.x];
        s_below[threadIdx.x] = bp->below[threadIdx.x];
        s_fill[threadIdx.x] = 0;
        // (found below; these values only stand if the counts were inconsistent)
        s_vstar[threadIdx.x] = 0xFFFFFFFFu;
        s_need2[threadIdx.x] = 1;
        s_cnt2[threadIdx.x] = 0;
        s_tk[threadIdx.x] = 0.0;
        s_tp[threadIdx.x] = 0;
    }
    __syncthreads();
    auto count_cls = [&](uint32_t cls, uint32_t p) {
        if (lds_counts) atomicAdd(&csel[cls * nb + p / kBS], 1u);
        else atomicAdd(&B.blockcnt[cls * B.nbs + p / kBS], 1u);
    };
    // (1) level-2 bins: one wave per distinct boundary bin (slot = its first
    // target); lane l holds bins 64 l .. 64 l + 63
    for (uint32_t i0 = wv; i0 < q; i0 += NT / 64) {
        if (i0 > 0 && s_bin[i0] == s_bin[i0 - 1]) continue;  // the same histogram
        uint32_t *hist = B.hist2 + i0 * kBins + lane * 64;
        constexpr int kC = 16;  // bins loaded at a time
        uint32_t sum = 0;
#pragma unroll
        for (int x0 = 0; x0 < 64; x0 += kC) {
            uint32_t h[kC];
#pragma unroll
            for (int x = 0; x < kC; ++x) h[x] = hist[x0 + x];
#pragma unroll
            for (int x = 0; x < kC; ++x) sum += h[x];
        }
        const uint32_t inc = wave_incl_scan(sum);
        const uint32_t pre = inc - sum;
        for (uint32_t i = i0; i < q && s_bin[i] == s_bin[i0]; ++i) {
            const uint32_t need1 = (i + 1) * N - s_below[i];
            if (pre < need1 && need1 <= pre + sum) {
                uint32_t cum = pre;
                for (int x0 = 0; x0 < 64; x0 += kC) {
                    uint32_t h[kC];
#pragma unroll
                    for (int x = 0; x < kC; ++x) h[x] = hist[x0 + x];
#pragma unroll
                    for (int x = 0; x < kC; ++x) {
                        if (cum < need1 && need1 <= cum + h[x]) {
                            s_vstar[i] = (s_bin[i] << 12) | (uint32_t)(lane * 64 + x0 + x);
                            s_need2[i] = need1 - cum;
                            s_cnt2[i] = h[x];
                        }
                        cum += h[x];
                    }
                }
            }
        }
        // cleared for the next batch (every read of this slot is above)
#pragma unroll
        for (int x = 0; x < 64; ++x) hist[x] = 0;
    }
    __syncthreads();
    // segments: every target whose level-2 bin fits gets its own stretch of
    // rk/rp (targets that share a level-2 bin share its members' counts:
    // only the first of them counts them)
    if (threadIdx.x == 0) {
        uint32_t off = 0, slow = 0;
        for (uint32_t i = 0; i < q; ++i) {
            const bool fits = off + s_cnt2[i] <= (uint32_t)kRankCap;
            s_fast[i] = fits ? 1u : 0u;
            s_seg[i] = off;
            if (fits) off += s_cnt2[i];
            else slow = 1u;
        }
        s_anyslow = slow;
    }
    __syncthreads();
    // (2) one pass over the candidates; the targets' level-2 values are
    // held in registers (a loop over LDS values would wait for an LDS read
    // per target and candidate), padded with values no candidate has
    uint32_t vst[kQMax];
#pragma unroll
    for (int i = 0; i < kQMax; ++i) vst[i] = (uint32_t)i < q ? s_vstar[i] : 0xFFFFFFFFu;
    for (uint32_t c0 = 0; c0 < ncand; c0 += NT * kBatch) {
        double kk[kBatch];
        uint32_t pp[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const uint32_t c = c0 + u * NT + threadIdx.x;
            // clamped, unconditional: the loads go out together
            const uint32_t cc = min(c, ncand - 1);
            kk[u] = B.ckey[cc];
            pp[u] = B.cpos[cc];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const uint32_t c = c0 + u * NT + threadIdx.x;
            const bool in = c < ncand;
            const uint32_t v = vmap(kk[u], base, vsh);
            // class: one past the last target whose level-2 value lies below
            // v (padding is never below; v < 2^24)
            uint32_t cls = 0;
            bool member = false;
#pragma unroll
            for (int i = 0; i < kQMax; ++i) {
                cls = v > vst[i] ? (uint32_t)i + 1u : cls;
                member |= v == vst[i];
            }
            member = member && in;
            if (member) {
                for (uint32_t i = 0; i < q; ++i)
                    if (v == s_vstar[i] && s_fast[i]) {
                        const uint32_t r = atomicAdd(&s_fill[i], 1u);
                        if (r < s_cnt2[i]) {
                            rk[s_seg[i] + r] = kk[u];
                            rp[s_seg[i] + r] = pp[u];
                        }
                    }
            }
            // the value alone decides every threshold (bins are monotone in
            // the key).  In LDS every lane adds its own candidate (one
            // instruction; lanes on one counter are serialised by the LDS
            // unit, cheaper than a wave loop over the distinct counters);
            // in global memory the wave adds up each (class, block) pair
            // first: one atomic per distinct pair
            const bool cnt_it = in && !member;
            const uint32_t key = cls * nb + pp[u] / kBS;
            if (lds_counts) {
                if (cnt_it) atomicAdd(&csel[key], 1u);
                continue;
            }
            uint64_t rest = __ballot(cnt_it);
            while (rest) {
                const int l0 = __ffsll((unsigned long long)rest) - 1;
                const uint32_t k0 = (uint32_t)__builtin_amdgcn_readlane((int)key, l0);
                const uint64_t m = __ballot(cnt_it && key == k0);
                if (lane == l0) atomicAdd(&B.blockcnt[(k0 / nb) * B.nbs + k0 % nb], (uint32_t)__popcll(m));
                rest &= ~m;
            }
        }
    }
    __syncthreads();
    // (3) exact ranks inside every segment (threads over all (target, member) pairs)
    uint32_t tot = 0;
    for (uint32_t i = 0; i < q; ++i) tot += s_fast[i] ? s_cnt2[i] : 0u;
    for (uint32_t x = threadIdx.x; x < tot; x += NT) {
        uint32_t i = 0;
        while (!(s_fast[i] && x >= s_seg[i] && x < s_seg[i] + s_cnt2[i])) ++i;
        const double kx = rk[x];
        const uint32_t px = rp[x];
        uint32_t r = 0;
        for (uint32_t y = s_seg[i]; y < s_seg[i] + s_cnt2[i]; ++y)
            r += (rk[y] < kx || (rk[y] == kx && rp[y] < px)) ? 1u : 0u;
        if (r == s_need2[i] - 1) {
            s_tk[i] = kx;
            s_tp[i] = px;
        }
    }
    __syncthreads();
    for (uint32_t i = 0; i < q; ++i) {
        if (s_fast[i]) continue;
        double thr_key;
        uint32_t thr_pos;
        slow_select<NT>(B.ckey, B.cpos, ncand, s_vstar[i], base, vsh, s_need2[i], h256, sh, &thr_key, &thr_pos);
        if (threadIdx.x == 0) {
            s_tk[i] = thr_key;
            s_tp[i] = thr_pos;
            B.st->fallback += 1;
        }
        __syncthreads();
    }
    auto exact_cls = [&](double k, uint32_t p) {
        uint32_t cls = 0;
        while (cls < q && !pair_le(k, p, s_tk[cls], s_tp[cls])) ++cls;
        return cls;
    };
    if (!s_anyslow) {
        // members of the fast segments, each counted once (by the first
        // target of its level-2 bin)
        for (uint32_t x = threadIdx.x; x < tot; x += NT) {
            uint32_t i = 0;
            while (!(s_fast[i] && x >= s_seg[i] && x < s_seg[i] + s_cnt2[i])) ++i;
            if (i == 0 || s_vstar[i - 1] != s_vstar[i]) count_cls(exact_cls(rk[x], rp[x]), rp[x]);
        }
    } else {
        // some level-2 bin was too large for LDS: its members (and all
        // others sharing a target's bin) are classified by one more pass
        for (uint32_t c = threadIdx.x; c < ncand; c += NT) {
            const double k = B.ckey[c];
            const uint32_t p = B.cpos[c];
            const uint32_t v = vmap(k, base, vsh);
            bool member = false;
            for (uint32_t i = 0; i < q; ++i) member = member || v == s_vstar[i];
            if (member) count_cls(exact_cls(k, p), p);
        }
    }
    // the landmark may move after the batch only if some attribute's
    // largest holder key is <= the last threshold's key (equality counted
    // as a move: a conservative test)
    if (threadIdx.x == 0) s_lch = (B.mk && !fixed) ? 0u : 1u;
    if (!lds_counts) __threadfence_block();
    __syncthreads();
    if (B.mk && !fixed && (int)threadIdx.x < B.d &&
        B.mk[(a & 1) * B.d + threadIdx.x] <= (unsigned long long)__double_as_longlong(s_tk[q - 1]))
        s_lch = 1u;
    // (4) per class, one wave scans the block counts, 8 chunks of 64 loaded
    // at a time (clamped, unconditional loads)
    for (uint32_t cls = wv; cls <= q; cls += NT / 64) {
        uint32_t carry = 0;
        for (uint32_t c0 = 0; c0 < nb; c0 += 64 * 8) {
            uint32_t v[8];
#pragma unroll
            for (int x = 0; x < 8; ++x) {
                const uint32_t sg = min(c0 + 64 * x + lane, nb - 1);
                v[x] = __hip_atomic_load(&B.blockcnt[cls * B.nbs + sg], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
#pragma unroll
            for (int x = 0; x < 8; ++x) {
                const uint32_t sg = c0 + 64 * x + lane;
                if (lds_counts) v[x] += csel[cls * nb + min(sg, nb - 1)];
                if (sg >= nb) v[x] = 0;
                const uint32_t inc = wave_incl_scan(v[x]);
                // read by the compaction blocks of this launch: stored at the
                // device's coherence point
                if (sg < nb)
                    __hip_atomic_store(&B.blockoff[cls * B.nbs + sg], carry + inc - v[x], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                carry += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < q) {
        __hip_atomic_store(&B.bp->thr_key[threadIdx.x], s_tk[threadIdx.x], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&B.bp->thr_pos[threadIdx.x], s_tp[threadIdx.x], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x == 0) {
        __hip_atomic_store(&B.bp->lchange, s_lch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        B.st->thr_key = s_tk[q - 1];  // centre of the next batch's key map
        B.act[t + q] = a + 1;
    }
    // the rounds inside the batch share its landmark
    if (B.landmarks)
        for (uint32_t x = threadIdx.x; x < (q - 1) * (uint32_t)B.d; x += NT)
            B.landmarks[((int64_t)t + 1) * B.d + x] = B.landmarks[(int64_t)t * B.d + x % B.d];
}

// Compaction of a batch (the rows of d = W * DQ attributes, early loads as in
// k_scatter_fast): every point's class is the first group whose threshold
// bounds it, or the rest; class c < q goes to subcluster t + c in ascending
// index, the rest to the next remaining list with its key; the minimum of
// the rest is folded into the next landmark when it may move.  all_sel:
// the last round, every remaining point to subcluster t.  FULL: every row of
// the block is requested before the classes are known (the landmark may
// move, so the rows that stay are needed too); otherwise only the rows that
// go to a subcluster are read, once their destinations are known.  The two
// forms are separate instantiations so that neither holds the other's
// registers.
struct ScatterLds {
    int32_t dst[kBS];  // >= 0: row within its subcluster; < 0: -(1 + slot) in rem_next
    uint8_t cls[kBS];
    unsigned long long wsum[kT / 64][2];
    double tk[kQMax];
    uint32_t tp[kQMax], off[kQMax + 1];
    uint32_t cmin[32];
};

template <int W, int DQ, bool FULL>
__device__ __forceinline__ void scatterm_body(const RoundBufs &B, ScatterLds &sm, uint32_t a,
                                              uint32_t t, uint32_t nrem, uint32_t N, int all_sel,
                                              int track_min, int fixed, uint32_t qn) {
    typedef typename VecT<W>::type V;
    constexpr int D = W * DQ;
    constexpr int per = kBS / kT;
    constexpr int RS = kT / DQ;
    constexpr int NV = kBS / RS;
    const int32_t *rem = t == 0 ? nullptr : B.rem[a & 1];
    int32_t *rem_next = B.rem[(a + 1) & 1];
    const double *keys = B.keys[a & 1];
    double *keys_next = B.keys[(a + 1) & 1];
    const uint32_t *Lcur = (t == 0 || fixed) ? nullptr : B.Lb + (a % 3) * D;
    uint32_t *Lnext = fixed ? nullptr : B.Lb + ((a + 1) % 3) * D;
    const uint32_t p0 = blockIdx.x * kBS;
    const uint32_t cnt = min(kBS, nrem - p0);
    const uint32_t last = p0 + cnt - 1;
    const int j = threadIdx.x % DQ;
    const uint32_t r0 = threadIdx.x / DQ;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t ridx[NV];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        const uint32_t p = min(p0 + r0 + u * RS, last);
        ridx[u] = rem ? rem[p] : (int32_t)p;
    }
    double kq[per];
    int32_t iq[per];
#pragma unroll
    for (int x = 0; x < per; ++x) {
        const uint32_t p = min(p0 + threadIdx.x * per + x, last);
        kq[x] = all_sel ? 0.0 : keys[p];
        iq[x] = rem ? rem[p] : (int32_t)p;
    }
    V v[NV];
    if (FULL) {
#pragma unroll
        for (int u = 0; u < NV; ++u) v[u] = ((const V *)(B.S + (int64_t)ridx[u] * D))[j];
    }
    // classes of the thread's positions, 4 bits each.  Most points stay:
    // one comparison with the last threshold (held in registers) settles
    // them, the others search the thresholds in order.
    uint32_t clsw = 0;
    const double tk_last = all_sel ? 0.0 : sm.tk[qn - 1];
    const uint32_t tp_last = all_sel ? 0u : sm.tp[qn - 1];
#pragma unroll
    for (int x = 0; x < per; ++x) {
        const uint32_t lp = threadIdx.x * per + x;
        uint32_t c = 0;
        if (!all_sel) {
            if (!pair_le(kq[x], p0 + lp, tk_last, tp_last)) c = qn;
            else
                while (c + 1 < qn && !pair_le(kq[x], p0 + lp, sm.tk[c], sm.tp[c])) ++c;
        }
        clsw |= (lp < cnt ? c : 15u) << (4 * x);
    }
    // per-class counts packed 12 bits a field, 5 fields a word (class c in
    // word c / 5); an exclusive scan of the two words over the block gives
    // every position its rank among the block's positions of its class
    auto packed = [&](int w) {
        unsigned long long pv = 0;
#pragma unroll
        for (int x = 0; x < per; ++x) {
            const uint32_t c = (clsw >> (4 * x)) & 15u;
            if (c != 15u && (int)(c / 5) == w) pv += 1ull << (12 * (c % 5));
        }
        return pv;
    };
    unsigned long long ex[2];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const unsigned long long xx = wave_incl_scan64(packed(w));
        if (lane == 63) sm.wsum[wv][w] = xx;
        ex[w] = xx;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        unsigned long long b0 = 0;
        for (int q = 0; q < wv; ++q) b0 += sm.wsum[q][w];
        ex[w] = b0 + ex[w] - packed(w);
    }
    const uint32_t stay_cap = nrem - (all_sel ? nrem : qn * N);
    const uint32_t sel_cap = all_sel ? nrem : N;
#pragma unroll
    for (int x = 0; x < per; ++x) {
        const uint32_t lp = threadIdx.x * per + x;
        if (lp < cnt) {
            const uint32_t c = (clsw >> (4 * x)) & 15u;
            uint32_t rk = 0;
#pragma unroll
            for (int w = 0; w < 2; ++w)
                if ((uint32_t)w == c / 5) {
                    rk = (uint32_t)(ex[w] >> (12 * (c % 5))) & 0xFFFu;
                    ex[w] += 1ull << (12 * (c % 5));
                }
            sm.cls[lp] = (uint8_t)c;
            if (c < qn) {
                // the guards only matter if the counts were inconsistent
                const uint32_t row = sm.off[c] + rk;
                const bool ok = row < sel_cap;
                sm.dst[lp] = ok ? (int32_t)row : INT32_MIN;
                if (ok) B.perm[((int64_t)t + c) * N + row] = iq[x];
            } else {
                const uint32_t slot = sm.off[qn] + rk;
                const bool ok = slot < stay_cap;
                sm.dst[lp] = ok ? -1 - (int32_t)slot : INT32_MIN;
                if (ok) {
                    rem_next[slot] = iq[x];
                    keys_next[slot] = kq[x];
                }
            }
        }
    }
    if (track_min && threadIdx.x < D) sm.cmin[threadIdx.x] = 0xFFFFFFFFu;
    __syncthreads();
    if (!FULL) {
        // every thread loads; a row that goes to no subcluster reads row 0
        // instead (one line for the whole grid), so the loads go out together
#pragma unroll
        for (int u = 0; u < NV; ++u) {
            const uint32_t rc = min(r0 + u * RS, cnt - 1);
            const int32_t row = sm.dst[rc] >= 0 ? ridx[u] : 0;
            v[u] = ((const V *)(B.S + (int64_t)row * D))[j];
        }
    }
    const bool fold = FULL && track_min;
    uint32_t mymin[W];
#pragma unroll
    for (int c = 0; c < W; ++c) mymin[c] = 0xFFFFFFFFu;
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        const uint32_t r = r0 + u * RS;
        if (r < cnt) {
            const int32_t dst = sm.dst[r];
            if (dst >= 0) {
                const int64_t prow = ((int64_t)t + sm.cls[r]) * N + dst;
                ((V *)(B.P + prow * D))[j] = v[u];
            } else if (fold && dst != INT32_MIN) {
#pragma unroll
                for (int c = 0; c < W; ++c) mymin[c] = min(mymin[c], ordered_bits(vget(v[u], c)));
            }
        }
    }
    if (fold) {
#pragma unroll
        for (int c = 0; c < W; ++c)
            if (mymin[c] != 0xFFFFFFFFu) atomicMin(&sm.cmin[j * W + c], mymin[c]);
        __syncthreads();
        if (threadIdx.x < D && sm.cmin[threadIdx.x] != 0xFFFFFFFFu)
            atomicMin(&Lnext[threadIdx.x], sm.cmin[threadIdx.x]);
    } else if (track_min && blockIdx.x == 0 && threadIdx.x < D) {
        // the landmark stays (every block takes this branch)
        Lnext[threadIdx.x] = Lcur ? Lcur[threadIdx.x] : ordered_bits(B.L0[threadIdx.x]);
    }
}

template <int W, int DQ>
__global__ __launch_bounds__(kT, W * DQ <= 16 ? 4 : 1) void k_scatterm(
    RoundBufs B, uint32_t t, uint32_t nrem, uint32_t N, int all_sel, int track_min, int lm_skip,
    int fixed) {
    constexpr int D = W * DQ;
    static_assert(kT % DQ == 0 && kBS % (kT / DQ) == 0, "attribute groups must tile the block");
    static_assert(kBS / kT <= 4 && kQMax + 1 <= 10, "class counts packed 5 x 12 bits per word, 2 words");
    static_assert(D <= 32, "row width of the early-load forms");
    const uint32_t a = B.act[t];
    if (a == kNoRound) return;
    __shared__ union {
        ScatterLds sc;
        Sel2Lds s2;
    } U;
    ScatterLds &sm = U.sc;
    if (!all_sel) {
        // The threshold step of the pass runs in block 0 of this launch (one
        // launch per pass fewer); the other blocks wait for its flag.  What
        // they read of it (thresholds, landmark flag, block offsets) is
        // stored and loaded at the device's coherence point; block 0 was
        // dispatched first, so the wait always ends (bounded all the same).
        if (blockIdx.x == 0) {
            sel2m_body<kT>(B, t, N, gridDim.x, fixed, a, U.s2);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (threadIdx.x == 0)
                __hip_atomic_store(&B.st->sel_done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (threadIdx.x == 0) {
            long long spins = 0;
            while (__hip_atomic_load(&B.st->sel_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1ll << 24)) {
                    atomicOr(B.err, 1);
                    break;
                }
            }
        }
        __syncthreads();
    }
    const uint32_t qn = all_sel ? 1u : B.bp->q;
    const uint32_t lch =
        all_sel ? 1u : __hip_atomic_load(&B.bp->lchange, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!all_sel && threadIdx.x < qn) {
        sm.tk[threadIdx.x] = __hip_atomic_load(&B.bp->thr_key[threadIdx.x], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
        sm.tp[threadIdx.x] = __hip_atomic_load(&B.bp->thr_pos[threadIdx.x], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x <= qn)
        sm.off[threadIdx.x] =
            all_sel ? (threadIdx.x == 0 ? blockIdx.x * kBS : 0u)
                    : __hip_atomic_load(&B.blockoff[threadIdx.x * B.nbs + blockIdx.x], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    // rows that stay are read only when the next landmark may move
    const bool full = !(lm_skip && !all_sel && (!track_min || lch == 0));
    if (full) scatterm_body<W, DQ, true>(B, sm, a, t, nrem, N, all_sel, track_min, fixed, qn);
    else scatterm_body<W, DQ, false>(B, sm, a, t, nrem, N, all_sel, track_min, fixed, qn);
    if (B.mk && !all_sel && blockIdx.x == 0 && threadIdx.x < D) B.mk[((a + 1) & 1) * D + threadIdx.x] = 0ull;
    if (!all_sel) {
        // the level-1 replicas and group counts were last read by the
        // candidate pass: clear them for the next batch, a slice per block
        constexpr uint32_t words = kRep * (kBins + kGroups);
        const uint32_t zs = (words + gridDim.x - 1) / gridDim.x;
        const uint32_t z0 = blockIdx.x * zs, z1 = min(words, z0 + zs);
        for (uint32_t i = z0 + threadIdx.x; i < z1; i += kT) B.hist1[i] = 0;
    }
}

typedef void (*ScatterMFn)(RoundBufs, uint32_t, uint32_t, uint32_t, int, int, int, int);

ScatterMFn scatterm_for(int d, bool vec4) {
    if (vec4) {
        switch (d) {
            case 4: return k_scatterm<4, 1>;
            case 8: return k_scatterm<4, 2>;
            case 16: return k_scatterm<4, 4>;
            case 32: return k_scatterm<4, 8>;
            default: return nullptr;
        }
    }
    switch (d) {
        case 1: return k_scatterm<1, 1>;
        case 2: return k_scatterm<1, 2>;
        case 4: return k_scatterm<1, 4>;
        case 8: return k_scatterm<1, 8>;
        default: return nullptr;
    }
}

// the landmark of the last round (a slot of its own) into the landmarks output
__global__ void k_land_last(RoundBufs B, uint32_t t, int fixed) {
    const uint32_t a = B.act[t];
    if (a == kNoRound) return;
    const int jj = blockIdx.x * blockDim.x + threadIdx.x;
    if (jj >= B.d) return;
    B.landmarks[(int64_t)t * B.d + jj] =
        (t == 0 || fixed) ? B.L0[jj] : ordered_float(B.Lb[(a % 3) * B.d + jj]);
}

__global__ void k_act_init(uint32_t *act, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) act[i] = i == 0 ? 0u : kNoRound;
}

}  // namespace


namespace {

struct SubBufs {
    double *keys;
    int32_t *rem0, *rem1;
    char *cand, *sel;
    float *land, *colmax;
    int *flag;
};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Layout of SC_SEL: the single-round state (SelState, level-1 replicas and
// group counts, level-2 bins, block counts and offsets), then the batch
// region (BatchPlan, act[T + 1], kQMax level-2 histograms, per-class block
// counts and offsets).
size_t sel_round_bytes(uint32_t nb_max) {
    return align256(256 + sizeof(uint32_t) * (2 * (size_t)kRep * kBins + 3 * (size_t)nb_max + 64));
}
size_t sel_batch_bytes(int64_t T, uint32_t nb_max) {
    return align256(sizeof(BatchPlan)) + align256(sizeof(uint32_t) * (size_t)(T + 1)) +
           sizeof(uint32_t) * ((size_t)kQMax * kBins + 2 * (size_t)(kQMax + 1) * nb_max) + 256;
}

// Scratch of one subclustering call (allocated before any capture).
void sub_requests(int64_t n, int32_t d, int64_t N, size_t *req) {
    auto need = [&](int slot, size_t b) { req[slot] = std::max(req[slot], b); };
    const uint32_t nb_max = (uint32_t)ceil_div(n, kBS);
    need(SC_KEYS, 2 * sizeof(double) * n);  // this round's keys and the carried ones
    need(SC_REM0, sizeof(int32_t) * n);
    need(SC_REM1, sizeof(int32_t) * n);
    need(SC_CAND, (sizeof(double) + sizeof(uint32_t)) * n + 64);
    need(SC_SEL, sel_round_bytes(nb_max) + sel_batch_bytes(ceil_div(n, std::max<int64_t>(N, 1)), nb_max));
    need(SC_LAND, sizeof(float) * (8 * (size_t)d + 64));
    need(SC_COLMAX, sizeof(float) * d + 64);
    need(SC_MM_FLAG, 256);
    need(SC_MM_PART, minmax_scratch_bytes(n, d));
}

subkm_status sub_alloc(subkm_ctx *ctx, int64_t n, int32_t d, int64_t N, SubBufs &b) {
    size_t req[SC_COUNT] = {};
    sub_requests(n, d, N, req);
    b.keys = (double *)ctx_scratch(ctx, SC_KEYS, req[SC_KEYS]);
    b.rem0 = (int32_t *)ctx_scratch(ctx, SC_REM0, req[SC_REM0]);
    b.rem1 = (int32_t *)ctx_scratch(ctx, SC_REM1, req[SC_REM1]);
    b.cand = (char *)ctx_scratch(ctx, SC_CAND, req[SC_CAND]);
    b.sel = (char *)ctx_scratch(ctx, SC_SEL, req[SC_SEL]);
    b.land = (float *)ctx_scratch(ctx, SC_LAND, req[SC_LAND]);
    b.colmax = (float *)ctx_scratch(ctx, SC_COLMAX, req[SC_COLMAX]);
    b.flag = (int *)ctx_scratch(ctx, SC_MM_FLAG, req[SC_MM_FLAG]);
    void *mm = ctx_scratch(ctx, SC_MM_PART, req[SC_MM_PART]);
    if (!b.keys || !b.rem0 || !b.rem1 || !b.cand || !b.sel || !b.land || !b.colmax || !b.flag || !mm)
        return SUBKM_ENOMEM;
    return SUBKM_OK;
}

// Every launch of one subclustering call in batches of rounds (row widths
// with the early-load kernels), in order, on ctx->stream.  The sequence is
// the same whatever the data: T round slots, each starting a batch or
// returning at once (act).
subkm_status sub_enqueue_batched(subkm_ctx *ctx, const SubBufs &b, const float *S, int64_t n,
                                 int32_t d, int64_t N, int32_t landmark_mode, int32_t metric,
                                 float *P, int32_t *perm, int64_t *offsets, float *landmarks) {
    const int64_t T = ceil_div(n, N);
    hipStream_t s = ctx->stream;
    const uint32_t nb_max = (uint32_t)ceil_div(n, kBS);
    const bool fixed = landmark_mode == 1;
    const bool vec4 = (d % 4) == 0 && ((uintptr_t)S % 16) == 0;
    const bool vec4p = vec4 && ((uintptr_t)P % 16) == 0;
    const ScatterMFn scat = scatterm_for(d, vec4p);
    RoundBufs B;
    std::memset(&B, 0, sizeof B);
    B.S = S;
    B.P = P;
    B.perm = perm;
    B.landmarks = landmarks;
    B.rem[0] = b.rem0;
    B.rem[1] = b.rem1;
    B.keys[0] = b.keys;
    B.keys[1] = b.keys + n;
    B.L0 = b.land;
    B.Lb = (uint32_t *)(b.land + d);
    B.mk = fixed ? nullptr : (unsigned long long *)(b.land + 4 * d);
    B.colmax = b.colmax;
    B.st = (SelState *)b.sel;
    uint32_t *hist1 = (uint32_t *)(b.sel + 256);
    B.hist1 = hist1;
    char *breg = b.sel + sel_round_bytes(nb_max);
    B.bp = (BatchPlan *)breg;
    B.act = (uint32_t *)(breg + align256(sizeof(BatchPlan)));
    B.hist2 = B.act + (align256(sizeof(uint32_t) * (size_t)(T + 1)) / sizeof(uint32_t));
    B.blockcnt = B.hist2 + (size_t)kQMax * kBins;
    B.blockoff = B.blockcnt + (size_t)(kQMax + 1) * nb_max;
    B.ckey = (double *)b.cand;
    B.cpos = (uint32_t *)(b.cand + sizeof(double) * n);
    B.nbs = nb_max;
    B.d = d;
    B.err = ctx->sticky;
    {
        const uint32_t nz1 = (uint32_t)(2 * kRep * kBins);
        hipLaunchKernelGGL(k_fill_u32, dim3(ceil_div(nz1, 256)), dim3(256), 0, s, hist1, nz1, 0u);
        SUBKM_LAUNCHED(ctx);
        const uint32_t nz2 = (uint32_t)(kQMax * kBins);
        hipLaunchKernelGGL(k_fill_u32, dim3(ceil_div(nz2, 256)), dim3(256), 0, s, B.hist2, nz2, 0u);
        SUBKM_LAUNCHED(ctx);
        hipLaunchKernelGGL(k_fill_u32, dim3(ceil_div(4 * d, 256)), dim3(256), 0, s,
                           (uint32_t *)(b.land + 4 * d), (uint32_t)(4 * d), 0u);
        SUBKM_LAUNCHED(ctx);
        hipLaunchKernelGGL(k_act_init, dim3(ceil_div(T + 1, 256)), dim3(256), 0, s, B.act,
                           (uint32_t)(T + 1));
        SUBKM_LAUNCHED(ctx);
        SUBKM_TRY(minmax_impl(ctx, S, n, d, b.land, b.colmax, b.flag));
        hipLaunchKernelGGL(k_offsets, dim3(ceil_div(T + 1, 256)), dim3(256), 0, s, offsets, T, N, n);
        SUBKM_LAUNCHED(ctx);
    }
    uint32_t nrem = (uint32_t)n;
    for (int64_t t = 0; t < T; ++t) {
        const uint32_t need = (uint32_t)std::min<int64_t>(N, nrem);
        const uint32_t nb = (uint32_t)ceil_div(nrem, kBS);
        const bool all = need == nrem;
        const bool track = !all && !fixed;
        if (!all) {
            {
                ProfScope pk(ctx, PK_KEYS);
                const int pp = keys_fast_pp_of(nrem);
                const KeysBFn kf = keys_b_for(metric, d, vec4, pp);
                hipLaunchKernelGGL(kf, dim3(ceil_div(nrem, (int64_t)kT * pp)), dim3(kT), 0, s, B,
                                   (uint32_t)t, nrem, fixed ? 1 : 0);
                SUBKM_LAUNCHED(ctx);
            }
            {
                ProfScope pc(ctx, PK_CAND);
                hipLaunchKernelGGL(k_candm, dim3(nb), dim3(kT), 0, s, B, (uint32_t)t, (uint32_t)T,
                                   nrem, (uint32_t)N);
                SUBKM_LAUNCHED(ctx);
            }

        } else if (landmarks) {
            hipLaunchKernelGGL(k_land_last, dim3(ceil_div(d, 256)), dim3(256), 0, s, B, (uint32_t)t,
                               fixed ? 1 : 0);
            SUBKM_LAUNCHED(ctx);
        }
        {
            ProfScope psc(ctx, PK_SCATTER);
            hipLaunchKernelGGL(scat, dim3(nb), dim3(kT), 0, s, B, (uint32_t)t, nrem, (uint32_t)N,
                               all ? 1 : 0, track ? 1 : 0, nrem >= kSkipMin ? 1 : 0, fixed ? 1 : 0);
            SUBKM_LAUNCHED(ctx);
        }
        nrem -= need;
    }
    return SUBKM_OK;
}

// Every launch of one subclustering call, in order, on ctx->stream.
subkm_status sub_enqueue(subkm_ctx *ctx, const SubBufs &b, const float *S, int64_t n, int32_t d,
                         int64_t N, int32_t landmark_mode, int32_t metric, float *P,
                         int32_t *perm, int64_t *offsets, float *landmarks, int64_t t0,
                         int64_t t1) {
    {
        const bool v4 = (d % 4) == 0 && ((uintptr_t)S % 16) == 0;
        const bool v4p = v4 && ((uintptr_t)P % 16) == 0;
        if (t0 == 0 && t1 == ceil_div(n, N) && scatterm_for(d, v4p) && keys_b_for(metric, d, v4, 1))
            return sub_enqueue_batched(ctx, b, S, n, d, N, landmark_mode, metric, P, perm, offsets,
                                       landmarks);
    }
    const int64_t T = ceil_div(n, N);
    hipStream_t s = ctx->stream;
    const uint32_t nb_max = (uint32_t)ceil_div(n, kBS);
    SelState *st = (SelState *)b.sel;
    // level-1 bin replicas, their group counts, then the level-2 bins
    uint32_t *hist1 = (uint32_t *)(b.sel + 256);
    uint32_t *hist2 = hist1 + kRep * (kBins + kGroups);
    uint32_t *blockcnt = hist1 + 2 * kRep * kBins;
    uint32_t *blockoff = blockcnt + nb_max;
    double *ckey = (double *)b.cand;
    uint32_t *cpos = (uint32_t *)(b.cand + sizeof(double) * n);
    float *L = b.land;  // first landmark (floats)
    // landmarks as ordered bits: round t >= 1 reads Lb[t % 3], folds the next
    // one into Lb[(t + 1) % 3] and compares with the previous one in
    // Lb[(t - 1) % 3] (round 0 saves its own there)
    uint32_t *Lb[3] = {(uint32_t *)(b.land + d), (uint32_t *)(b.land + 2 * d),
                       (uint32_t *)(b.land + 3 * d)};
    // keys of round t in Kb[t & 1]; the compaction carries the keys of the
    // points that stay into Kb[(t + 1) & 1]
    double *Kb[2] = {b.keys, b.keys + n};
    // per attribute, the largest key among the points holding the landmark
    // value (binary64 bits): round t in MK[t & 1]
    unsigned long long *MK[2] = {(unsigned long long *)(b.land + 4 * d),
                                 (unsigned long long *)(b.land + 4 * d) + d};
    int32_t *rem0 = b.rem0, *rem1 = b.rem1;
    const float *colmax = b.colmax;

    if (t0 == 0) {
        // histograms start at zero (the compaction and k_sel2 re-zero them)
        const uint32_t nzero = (uint32_t)(2 * kRep * kBins);
        hipLaunchKernelGGL(k_fill_u32, dim3(ceil_div(nzero, 256)), dim3(256), 0, s, hist1, nzero, 0u);
        SUBKM_LAUNCHED(ctx);
        hipLaunchKernelGGL(k_fill_u32, dim3(ceil_div(4 * d, 256)), dim3(256), 0, s,
                           (uint32_t *)MK[0], (uint32_t)(4 * d), 0u);
        SUBKM_LAUNCHED(ctx);
        // first landmark: attribute-wise minimum of all points; column maxima bound the keys
        SUBKM_TRY(minmax_impl(ctx, S, n, d, L, b.colmax, b.flag));
        hipLaunchKernelGGL(k_offsets, dim3(ceil_div(T + 1, 256)), dim3(256), 0, s, offsets, T, N, n);
        SUBKM_LAUNCHED(ctx);
    }

    const bool fixed = landmark_mode == 1;
    const bool vec4 = (d % 4) == 0 && ((uintptr_t)S % 16) == 0;
    const bool vec4p = vec4 && ((uintptr_t)P % 16) == 0;
    const ScatterFastFn scat_fast = scatter_fast_for(d, vec4p);
    // keys are carried from round to round when both early-load kernels run
    const bool carry = scat_fast && keys_fast_for(metric, d, vec4, 1);
    // the keys pass records the holder keys; the compaction then skips the
    // rows that stay in rounds whose landmark surely stays
    const bool lm_track = carry && !fixed;
    int32_t *cur = nullptr;  // round 0 reads the points through the identity
    int32_t *nxt = rem0;
    uint32_t nrem = (uint32_t)n;
    const size_t dyn_d = sizeof(float) * d;
    for (int64_t t = 0; t < t1; ++t) {
        const uint32_t need = (uint32_t)std::min<int64_t>(N, nrem);
        const uint32_t nb = (uint32_t)ceil_div(nrem, kBS);
        const bool all = need == nrem;
        float *lm_t = landmarks ? landmarks + t * d : nullptr;
        const bool track = !all && !fixed;
        const uint32_t *Lcur = (t == 0 || fixed) ? nullptr : Lb[t % 3];
        uint32_t *Lnext = track ? Lb[(t + 1) % 3] : nullptr;
        double *keys = Kb[t & 1];
        double *keys_next = carry && !all ? Kb[(t + 1) & 1] : nullptr;
        const int reuse = (!carry || t == 0) ? 0 : fixed ? 2 : 1;
        const uint32_t *Lprev = reuse == 1 ? Lb[(t + 2) % 3] : nullptr;
        uint32_t *Lsave = (carry && t == 0 && !fixed) ? Lb[0] : nullptr;
        unsigned long long *mk = lm_track ? MK[t & 1] : nullptr;
        unsigned long long *mk_other = lm_track ? MK[(t + 1) & 1] : nullptr;
        if (t < t0) {
            // rounds of earlier segments: only their host-side bookkeeping
            if (!all && !cur) cur = rem1;
            nrem -= need;
            int32_t *written = nxt;
            nxt = (written == rem0) ? rem1 : rem0;
            cur = written;
            continue;
        }
        if (!all) {
            if (!cur) {
                hipLaunchKernelGGL(k_iota, dim3(ceil_div(nrem, 256)), dim3(256), 0, s, rem1, nrem);
                SUBKM_LAUNCHED(ctx);
                cur = rem1;
            }
            {
                ProfScope pk(ctx, PK_KEYS);
                const int pp = keys_fast_pp_of(nrem);
                const KeysFastFn kf = keys_fast_for(metric, d, vec4, pp);
                if (kf) {
                    hipLaunchKernelGGL(kf, dim3(ceil_div(nrem, (int64_t)kT * pp)), dim3(kT), 0, s,
                                       S, cur, nrem, L, Lcur, Lnext, colmax, keys, hist1, st, lm_t,
                                       t > 0 ? 1 : 0, reuse, Lprev, Lsave, mk, mk_other);
                } else {
                    const int64_t grid = std::min<int64_t>(ceil_div(nrem, kT), 512);
                    hipLaunchKernelGGL(metric ? k_keys<1> : k_keys<0>, dim3(grid), dim3(kT), dyn_d,
                                       s, S, d, cur, nrem, L, Lcur, Lnext, colmax, keys, hist1, st,
                                       lm_t, vec4 ? 1 : 0, t > 0 ? 1 : 0);
                }
                SUBKM_LAUNCHED(ctx);
            }
            {
                ProfScope pc(ctx, PK_CAND);
                hipLaunchKernelGGL(k_cand, dim3(nb), dim3(kT), 0, s, keys, nrem, need, st, ckey,
                                   cpos, hist1, hist2, blockcnt);
                SUBKM_LAUNCHED(ctx);
            }
            hipLaunchKernelGGL(k_sel2, dim3(1), dim3(kST), 0, s, need, st, ckey, cpos, nb, hist2,
                               blockcnt, blockoff, mk, d);
            SUBKM_LAUNCHED(ctx);
        } else if (lm_t) {
            if (Lcur) hipLaunchKernelGGL(k_bits_to_f32, dim3(ceil_div(d, 256)), dim3(256), 0, s, lm_t, Lcur, d);
            else hipLaunchKernelGGL(k_copy_f32, dim3(ceil_div(d, 256)), dim3(256), 0, s, lm_t, L, d);
            SUBKM_LAUNCHED(ctx);
        }
        {
            ProfScope psc(ctx, PK_SCATTER);
            if (scat_fast)
                hipLaunchKernelGGL(scat_fast, dim3(nb), dim3(kT), 0, s, S, cur, keys, nrem, need,
                                   st, blockoff, all ? 1 : 0, track ? 1 : 0, P, perm, t * N, nxt,
                                   Lnext, keys_next, hist1, nrem >= kSkipMin ? 1 : 0, Lcur, L,
                                   all ? nullptr : mk_other);
            else
                hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kT), dyn_d, s, S, d, cur, keys, nrem,
                                   need, st, blockoff, all ? 1 : 0, track ? 1 : 0, P, perm, t * N,
                                   nxt, Lnext, vec4p ? 1 : 0, hist1);
            SUBKM_LAUNCHED(ctx);
        }
        nrem -= need;
        int32_t *written = nxt;
        nxt = (written == rem0) ? rem1 : rem0;
        cur = written;
    }
    return SUBKM_OK;
}

}  // namespace

// Rounds [t0, t1) of the sequence (3 + about 4 T launches in all) are
// captured once into a HIP graph per (segment, inputs, outputs, sizes,
// buffers) and replayed, which removes the launch gaps between the many short
// kernels.  The graphs hold kernel nodes only.
subkm_status subcluster_segment(subkm_ctx *ctx, const float *S, int64_t n, int32_t d, int64_t N,
                                int32_t landmark_mode, int32_t metric, float *P, int32_t *perm,
                                int64_t *offsets, float *landmarks, int64_t t0, int64_t t1,
                                int32_t seg) {
    SubBufs b;
    SUBKM_TRY(sub_alloc(ctx, n, d, N, b));
    // every input of the captured sequence, one word each
    const uint64_t key[subkm_ctx::kGraphKeyWords] = {
        (uint64_t)(uintptr_t)S, (uint64_t)n, (uint64_t)d, (uint64_t)N,
        (uint64_t)landmark_mode | ((uint64_t)metric << 8) | ((uint64_t)seg << 16),
        (uint64_t)(uintptr_t)P, (uint64_t)(uintptr_t)perm, (uint64_t)(uintptr_t)offsets,
        (uint64_t)(uintptr_t)landmarks, (uint64_t)(uintptr_t)b.keys, (uint64_t)(uintptr_t)b.rem0,
        (uint64_t)(uintptr_t)b.rem1, (uint64_t)(uintptr_t)b.cand, (uint64_t)(uintptr_t)b.sel,
        (uint64_t)(uintptr_t)b.land, (uint64_t)(uintptr_t)b.colmax, (uint64_t)(uintptr_t)b.flag,
        (uint64_t)(uintptr_t)ctx->scratch[SC_MM_PART].ptr, (uint64_t)t0, (uint64_t)t1, 0};
    subkm_ctx::GraphCache *gp = nullptr;
    for (auto &e : ctx->subg)
        if (e.valid && std::memcmp(e.key, key, sizeof key) == 0) {
            gp = &e;
            break;
        }
    if (!gp) {
        // a free entry, else the least recently used one
        if (ctx->subg.size() < subkm_ctx::kGraphCacheMax) {
            ctx->subg.emplace_back();
            gp = &ctx->subg.back();
        } else {
            gp = &ctx->subg[0];
            for (auto &e : ctx->subg)
                if (e.stamp < gp->stamp) gp = &e;
        }
    }
    auto &g = *gp;
    g.stamp = ++ctx->subg_clock;
    if (!(g.valid && std::memcmp(g.key, key, sizeof key) == 0)) {
        if (g.exec) {
            // an earlier launch of it may still be running
            SUBKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
            hipGraphExecDestroy(g.exec);
            g.exec = nullptr;
        }
        g.valid = false;
        if (!ctx->cap_stream)
            SUBKM_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        hipStream_t user = ctx->stream;
        const bool prof = ctx->prof_on;
        ctx->stream = ctx->cap_stream;
        ctx->prof_on = false;
        hipGraph_t graph = nullptr;
        subkm_status st = SUBKM_OK;
        hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
            st = sub_enqueue(ctx, b, S, n, d, N, landmark_mode, metric, P, perm, offsets,
                             landmarks, t0, t1);
            e = hipStreamEndCapture(ctx->cap_stream, &graph);
        }
        ctx->stream = user;
        ctx->prof_on = prof;
        if (st != SUBKM_OK) {
            if (graph) hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return set_err(ctx, SUBKM_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g.exec = nullptr;
            return set_err(ctx, SUBKM_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
        }
        std::memcpy(g.key, key, sizeof key);
        g.valid = true;
    }
    ProfScope ps(ctx, PK_SUBCLUSTER);
    SUBKM_HIP(ctx, hipGraphLaunch(g.exec, ctx->stream));
    return SUBKM_OK;
}

subkm_status subcluster_impl(subkm_ctx *ctx, const float *S, int64_t n, int32_t d, int64_t N,
                             int32_t landmark_mode, int32_t metric, float *P, int32_t *perm,
                             int64_t *offsets, float *landmarks) {
    return subcluster_segment(ctx, S, n, d, N, landmark_mode, metric, P, perm, offsets,
                              landmarks, 0, ceil_div(n, N), 0);
}

// Selection passes of the last subclustering call with these arguments on
// ctx (reads its scratch once the stream has drained): a pass serves one
// round, or a batch of rounds that share a landmark; the last round takes
// every point left and needs none.  Without the batched kernels every round
// but the last selects on its own.
subkm_status subcluster_selections(subkm_ctx *ctx, const float *S, const float *P, int64_t n,
                                   int32_t d, int64_t N, int32_t metric, int64_t *out) {
    const int64_t T = ceil_div(n, N);
    *out = T > 1 ? T - 1 : 0;
    const bool v4 = (d % 4) == 0 && ((uintptr_t)S % 16) == 0;
    const bool v4p = v4 && ((uintptr_t)P % 16) == 0;
    if (T <= 1 || !scatterm_for(d, v4p) || !keys_b_for(metric, d, v4, 1)) return SUBKM_OK;
    SubBufs b;
    SUBKM_TRY(sub_alloc(ctx, n, d, N, b));
    const uint32_t nb_max = (uint32_t)ceil_div(n, kBS);
    // act[T - 1]: batches before the last round, which always has a slot of its own
    const uint32_t *act =
        (const uint32_t *)(b.sel + sel_round_bytes(nb_max) + align256(sizeof(BatchPlan)));
    uint32_t a = 0;
    SUBKM_HIP(ctx, hipMemcpyAsync(&a, act + (T - 1), sizeof a, hipMemcpyDeviceToHost, ctx->stream));
    SUBKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *out = a;
    return SUBKM_OK;
}

void subcluster_scratch_requests(int64_t n, int32_t d, int64_t N, size_t *req) {
    sub_requests(n, d, N, req);
}
