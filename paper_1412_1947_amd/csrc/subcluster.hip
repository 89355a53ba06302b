// Equal sized subclustering (Sec. II, Algorithm 1 steps 2, 3 and 5), applied
// round after round to the points left over.
//
// Every round is three launches over the remaining points, with no host
// round trip (the threshold lives in device memory):
//
//   k_keys     binary64 key of every remaining point (its squared distance to
//              the landmark, attributes left to right, no FMA) + a 4096-bin
//              histogram of a monotone 24-bit image v(key) of the key.  The
//              last block to finish scans the histogram and finds the bin a*
//              that holds the N-th smallest key.
//   k_cand     appends the points of bin a* to a candidate list and
//              histograms their low 12 bits of v; counts per compaction block
//              the points surely selected (bin < a*).  The last block finds
//              the sub-bin, ranks the few candidates that share the whole v
//              exactly by (key, position) and so obtains the threshold pair
//              (key*, pos*); then it turns block counts into block offsets.
//   k_scatter  stable compaction: a point is selected iff (key, pos) <=
//              (key*, pos*); selected rows go to P / perm in ascending index,
//              the rest to the next remaining list, whose attribute-wise
//              minimum (the next landmark, Algorithm 1 step 2) is reduced in
//              the same pass.
//
// Positions in the remaining list are in ascending original index, so the
// index tie-break of the selection is a tie-break on positions.
#include "internal.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace {

constexpr int kT = 512;           // threads per block in every kernel here
constexpr int kBins = 4096;       // histogram bins per level
constexpr uint32_t kBS = 2048;    // positions per compaction block
constexpr int kRankCap = 2048;    // candidates ranked in LDS by the last block
constexpr uint32_t kVMax = 0xFFFFFFu;

struct SelState {
    uint32_t done1, done2, done3;
    uint32_t base;     // v-map offset of this round
    uint32_t astar, below1, cnt1;
    uint32_t bstar, below2, cnt2, need2;
    uint32_t ncand;
    uint32_t thr_pos;
    uint32_t fallback;  // rounds that needed the slow exact path
    uint32_t pad[2];
    double thr_key;
};

// Monotone non-decreasing map of a non-negative key to [0, 2^24): float32
// rounding (monotone), its bit pattern without the 4 lowest bits, offset so
// that the largest possible key lands in the top bin, clamped at both ends.
__device__ __forceinline__ uint32_t vmap(double key, uint32_t base) {
    uint32_t u = __float_as_uint((float)key) >> 4;
    uint32_t v = u > base ? u - base : 0u;
    return v > kVMax ? kVMax : v;
}

__device__ __forceinline__ uint32_t vbase_of(double bound) {
    uint32_t top = __float_as_uint((float)bound) >> 4;
    return top > kVMax ? top - kVMax : 0u;
}

__device__ __forceinline__ bool pair_le(double ka, uint32_t pa, double kb, uint32_t pb) {
    return ka < kb || (ka == kb && pa <= pb);
}

// Exclusive scan of one value per thread over a kT-thread block.  Returns
// the prefix; *total receives the block sum.  `tmp` holds kT/64 words.
__device__ uint32_t block_scan(uint32_t v, uint32_t *tmp, uint32_t *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) tmp[wave] = x;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
    for (int w = 0; w < kT / 64; ++w) {
        uint32_t s = tmp[w];
        if (w < wave) wbase += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wbase + x - v;
}

// Find the bin holding the need-th element (1-based) of a kBins histogram in
// global memory.  Every thread returns the same (bin, below, count).
__device__ void find_bin(const uint32_t *hist, uint32_t need, uint32_t *sh, uint32_t *tmp,
                         uint32_t *bin, uint32_t *below, uint32_t *count) {
    constexpr int per = kBins / kT;
    if (threadIdx.x == 0) sh[0] = sh[1] = sh[2] = 0;
    uint32_t h[per], s = 0;
#pragma unroll
    for (int q = 0; q < per; ++q) {
        h[q] = __hip_atomic_load(hist + threadIdx.x * per + q, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        s += h[q];
    }
    uint32_t tot;
    uint32_t cum = block_scan(s, tmp, &tot);
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

// "Am I the last block to finish?"  Publishes this block's global writes
// first; the last block then sees every other block's writes.
__device__ bool last_block(uint32_t *counter, uint32_t *flag_sh) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) *flag_sh = atomicAdd(counter, 1u) == gridDim.x - 1;
    __syncthreads();
    bool last = *flag_sh != 0;
    if (last) __threadfence();
    return last;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kT) void k_keys(const float *__restrict__ S, int d,
                                             const int32_t *__restrict__ rem, uint32_t nrem,
                                             uint32_t need, const float *__restrict__ L,
                                             const float *__restrict__ colmax,
                                             double *__restrict__ keys, uint32_t *hist1,
                                             SelState *st, float *landmarks_t, int vec4) {
    extern __shared__ float sL[];  // d floats
    __shared__ uint32_t h[kBins];
    __shared__ uint32_t sh[4], tmp[kT / 64], s_base, s_last;
    for (int i = threadIdx.x; i < kBins; i += kT) h[i] = 0;
    for (int j = threadIdx.x; j < d; j += kT) sL[j] = L[j];
    if (threadIdx.x == 0) {
        // upper bound of any key of this round: sum_j (max_j - L_j)^2
        double b = 0.0;
        for (int j = 0; j < d; ++j) {
            double q = (double)colmax[j] - (double)L[j];
            b = b + q * q;
        }
        s_base = vbase_of(b);
    }
    __syncthreads();
    if (blockIdx.x == 0 && landmarks_t)
        for (int j = threadIdx.x; j < d; j += kT) landmarks_t[j] = sL[j];
    const uint32_t base = s_base;
    for (uint32_t p = blockIdx.x * kT + threadIdx.x; p < nrem; p += gridDim.x * kT) {
        const float *row = S + (int64_t)rem[p] * d;
        double key = 0.0;
        if (vec4) {
            const float4 *r4 = (const float4 *)row;
            for (int j4 = 0; j4 < (d >> 2); ++j4) {
                float4 x = r4[j4];
                double q;
                q = (double)x.x - (double)sL[4 * j4 + 0]; key = key + q * q;
                q = (double)x.y - (double)sL[4 * j4 + 1]; key = key + q * q;
                q = (double)x.z - (double)sL[4 * j4 + 2]; key = key + q * q;
                q = (double)x.w - (double)sL[4 * j4 + 3]; key = key + q * q;
            }
        } else {
            for (int j = 0; j < d; ++j) {
                double q = (double)row[j] - (double)sL[j];
                key = key + q * q;
            }
        }
        keys[p] = key;
        atomicAdd(&h[vmap(key, base) >> 12], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += kT)
        if (h[i]) atomicAdd(&hist1[i], h[i]);
    if (!last_block(&st->done1, &s_last)) return;
    uint32_t a, below, cnt;
    find_bin(hist1, need, sh, tmp, &a, &below, &cnt);
    for (int i = threadIdx.x; i < kBins; i += kT) hist1[i] = 0;
    if (threadIdx.x == 0) {
        st->base = base;
        st->astar = a;
        st->below1 = below;
        st->cnt1 = cnt;
        st->ncand = 0;
        st->done1 = 0;
    }
}

// Exact selection of the need2-th smallest (key, pos) among the candidates
// whose v equals vstar, when there are too many of them to rank in LDS: a
// most-significant-digit radix select over the 96-bit pair, 8 bits a pass.
__device__ void slow_select(const double *ckey, const uint32_t *cpos, uint32_t ncand,
                            uint32_t vstar, uint32_t base, uint32_t need, uint32_t *hist256,
                            uint32_t *sh, uint32_t *tmp, double *thr_key, uint32_t *thr_pos) {
    uint64_t kpre = 0;
    uint32_t ppre = 0;
    for (int pass = 0; pass < 12; ++pass) {
        for (int i = threadIdx.x; i < 256; i += kT) hist256[i] = 0;
        __syncthreads();
        for (uint32_t c = threadIdx.x; c < ncand; c += kT) {
            double k = ckey[c];
            if (vmap(k, base) != vstar) continue;
            uint64_t kb = (uint64_t)__double_as_longlong(k);
            uint32_t p = cpos[c];
            bool match;
            uint32_t dig;
            if (pass < 8) {
                int sh_hi = 64 - 8 * pass;  // bits above the current digit
                match = pass == 0 || (kb >> sh_hi) == (kpre >> sh_hi);
                dig = (uint32_t)(kb >> (56 - 8 * pass)) & 255u;
            } else {
                int q = pass - 8;
                match = kb == kpre && (q == 0 || (p >> (32 - 8 * q)) == (ppre >> (32 - 8 * q)));
                dig = (p >> (24 - 8 * q)) & 255u;
            }
            if (match) atomicAdd(&hist256[dig], 1u);
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
        uint32_t b = sh[0];
        need -= sh[1];
        if (pass < 8) kpre |= (uint64_t)b << (56 - 8 * pass);
        else ppre |= b << (24 - 8 * (pass - 8));
        __syncthreads();
    }
    *thr_key = __longlong_as_double((long long)kpre);
    *thr_pos = ppre;
}

__global__ __launch_bounds__(kT) void k_cand(const double *__restrict__ keys, uint32_t nrem,
                                             uint32_t need, SelState *st,
                                             double *__restrict__ ckey,
                                             uint32_t *__restrict__ cpos, uint32_t *hist2,
                                             uint32_t *blockcnt, uint32_t *blockoff,
                                             uint32_t nblocks) {
    __shared__ uint32_t h[kBins];
    __shared__ uint32_t sh[4], tmp[kT / 64], s_last, s_red[kT / 64];
    __shared__ double rk[kRankCap];
    __shared__ uint32_t rp[kRankCap];
    __shared__ uint32_t s_n;
    for (int i = threadIdx.x; i < kBins; i += kT) h[i] = 0;
    __syncthreads();
    const uint32_t astar = st->astar, base = st->base;
    const int lane = threadIdx.x & 63;
    uint32_t below = 0;
    const uint32_t p0 = blockIdx.x * kBS;
    for (uint32_t q = threadIdx.x; q < kBS; q += kT) {
        const uint32_t p = p0 + q;
        bool in = p < nrem;
        double k = in ? keys[p] : 0.0;
        uint32_t v = in ? vmap(k, base) : 0u;
        uint32_t a = v >> 12;
        below += (in && a < astar) ? 1u : 0u;
        bool c = in && a == astar;
        uint64_t m = __ballot(c);
        if (m) {
            uint32_t cnt = (uint32_t)__popcll(m);
            uint32_t first = (uint32_t)__ffsll((unsigned long long)m) - 1;
            uint32_t slot0 = 0;
            if (lane == (int)first) slot0 = atomicAdd(&st->ncand, cnt);
            slot0 = __shfl(slot0, first, 64);
            if (c) {
                uint32_t rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
                ckey[slot0 + rank] = k;
                cpos[slot0 + rank] = p;
                atomicAdd(&h[v & 0xFFFu], 1u);
            }
        }
    }
    // block total of surely-selected points
    for (int o = 32; o > 0; o >>= 1) below += __shfl_xor(below, o, 64);
    if (lane == 0) s_red[threadIdx.x >> 6] = below;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kT / 64; ++w) s += s_red[w];
        blockcnt[blockIdx.x] = s;
    }
    for (int i = threadIdx.x; i < kBins; i += kT)
        if (h[i]) atomicAdd(&hist2[i], h[i]);
    if (!last_block(&st->done2, &s_last)) return;

    // ---- last block: the exact threshold ----
    const uint32_t need1 = need - st->below1;
    uint32_t b, below2, cnt2;
    find_bin(hist2, need1, sh, tmp, &b, &below2, &cnt2);
    const uint32_t need2 = need1 - below2;
    const uint32_t vstar = (astar << 12) | b;
    const uint32_t ncand = __hip_atomic_load(&st->ncand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double thr_key;
    uint32_t thr_pos;
    if (cnt2 <= (uint32_t)kRankCap) {
        if (threadIdx.x == 0) s_n = 0;
        __syncthreads();
        for (uint32_t c = threadIdx.x; c < ncand; c += kT) {
            double k = ckey[c];
            if (vmap(k, base) == vstar) {
                uint32_t s = atomicAdd(&s_n, 1u);
                if (s < (uint32_t)kRankCap) {
                    rk[s] = k;
                    rp[s] = cpos[c];
                }
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cnt2; i += kT) {
            const double ki = rk[i];
            const uint32_t pi = rp[i];
            uint32_t r = 0;
            for (uint32_t j = 0; j < cnt2; ++j) r += (rk[j] < ki || (rk[j] == ki && rp[j] < pi)) ? 1u : 0u;
            if (r == need2 - 1) sh[0] = i;
        }
        __syncthreads();
        thr_key = rk[sh[0]];
        thr_pos = rp[sh[0]];
        __syncthreads();
    } else {
        slow_select(ckey, cpos, ncand, vstar, base, need2, h, sh, tmp, &thr_key, &thr_pos);
        if (threadIdx.x == 0) st->fallback += 1;
    }
    // selected candidates join their block's count
    for (uint32_t c = threadIdx.x; c < ncand; c += kT) {
        if (pair_le(ckey[c], cpos[c], thr_key, thr_pos)) atomicAdd(&blockcnt[cpos[c] / kBS], 1u);
    }
    __threadfence_block();
    __syncthreads();
    // exclusive scan of the block counts -> selected-row offset of every block
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < nblocks; c0 += kT) {
        uint32_t i = c0 + threadIdx.x;
        uint32_t v = i < nblocks ? __hip_atomic_load(&blockcnt[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        uint32_t tot;
        uint32_t pre = block_scan(v, tmp, &tot);
        if (i < nblocks) blockoff[i] = carry + pre;
        carry += tot;
    }
    for (int i = threadIdx.x; i < kBins; i += kT) hist2[i] = 0;
    if (threadIdx.x == 0) {
        st->bstar = b;
        st->below2 = below2;
        st->cnt2 = cnt2;
        st->need2 = need2;
        st->thr_key = thr_key;
        st->thr_pos = thr_pos;
        st->done2 = 0;
    }
}

// ---------------------------------------------------------------------------
// Stable compaction of one block of kBS positions.  all_sel: every remaining
// point is selected (last round).  track_min: reduce the attribute-wise
// minimum of the points that stay (the next landmark).
__global__ __launch_bounds__(kT) void k_scatter(const float *__restrict__ S, int d,
                                                const int32_t *__restrict__ rem,
                                                const double *__restrict__ keys, uint32_t nrem,
                                                const SelState *st,
                                                const uint32_t *__restrict__ blockoff,
                                                int all_sel, int track_min, float *__restrict__ P,
                                                int32_t *__restrict__ perm, int64_t off_t,
                                                int32_t *__restrict__ rem_next, uint32_t *Lmin,
                                                float *L, float *landmarks_next,
                                                uint32_t *done3, uint32_t need) {
    __shared__ int32_t s_src[kBS];
    __shared__ int32_t s_dst[kBS];  // >= 0: P row; < 0: -(1 + slot) in rem_next
    __shared__ uint32_t tmp[kT / 64], s_last;
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
    // flags of this thread's `per` consecutive positions
    bool sel[per];
    uint32_t nsel = 0;
#pragma unroll
    for (int q = 0; q < per; ++q) {
        uint32_t lp = threadIdx.x * per + q;
        bool in = lp < cnt;
        bool s = false;
        if (in) s = all_sel || pair_le(keys[p0 + lp], p0 + lp, thr_key, thr_pos);
        sel[q] = s;
        nsel += s ? 1u : 0u;
    }
    uint32_t tot;
    uint32_t pre = block_scan(nsel, tmp, &tot);
    const uint32_t sel_base = all_sel ? p0 : blockoff[blockIdx.x];
    const uint32_t stay_base = p0 - sel_base;
    uint32_t si = pre, ti = threadIdx.x * per - pre;
#pragma unroll
    for (int q = 0; q < per; ++q) {
        uint32_t lp = threadIdx.x * per + q;
        if (lp < cnt) {
            int32_t idx = rem ? rem[p0 + lp] : (int32_t)(p0 + lp);
            s_src[lp] = idx;
            // the guards only matter if the selection counts were inconsistent
            if (sel[q]) {
                uint32_t row = sel_base + si++;
                bool ok = row < need;
                s_dst[lp] = ok ? (int32_t)row : INT32_MIN;
                if (ok) perm[off_t + row] = idx;
            } else {
                uint32_t slot = stay_base + ti++;
                bool ok = slot < nrem - need;
                s_dst[lp] = ok ? -1 - (int32_t)slot : INT32_MIN;
                if (ok) rem_next[slot] = idx;
            }
        }
    }
    const bool fixed_col = (kT % d) == 0;
    if (track_min && !fixed_col)
        for (int j = threadIdx.x; j < d; j += kT) s_cmin[j] = 0xFFFFFFFFu;
    __syncthreads();
    // rows: copy the selected ones, reduce the minimum of the others
    uint32_t my_min = 0xFFFFFFFFu;
    const int64_t total = (int64_t)cnt * d;
    const bool need_rows = track_min || tot > 0;
    if (need_rows) {
        for (int64_t e = threadIdx.x; e < total; e += kT) {
            uint32_t r = (uint32_t)(e / d);
            uint32_t j = (uint32_t)(e - (int64_t)r * d);
            int32_t dst = s_dst[r];
            if (dst == INT32_MIN) continue;
            if (dst >= 0) {
                P[((int64_t)off_t + dst) * d + j] = S[(int64_t)s_src[r] * d + j];
            } else if (track_min) {
                uint32_t o = ordered_bits(S[(int64_t)s_src[r] * d + j]);
                if (fixed_col) my_min = min(my_min, o);
                else atomicMin(&s_cmin[j], o);
            }
        }
    }
    if (track_min) {
        if (fixed_col) {
            s_min[threadIdx.x] = my_min;
            __syncthreads();
            for (int j = threadIdx.x; j < d; j += kT) {
                uint32_t m = 0xFFFFFFFFu;
                for (int t = j; t < kT; t += d) m = min(m, s_min[t]);
                if (m != 0xFFFFFFFFu) atomicMin(&Lmin[j], m);
            }
        } else {
            __syncthreads();
            for (int j = threadIdx.x; j < d; j += kT)
                if (s_cmin[j] != 0xFFFFFFFFu) atomicMin(&Lmin[j], s_cmin[j]);
        }
    }
    if (!last_block(done3, &s_last)) return;
    if (track_min) {
        for (int j = threadIdx.x; j < d; j += kT) {
            uint32_t m = __hip_atomic_load(&Lmin[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            float f = ordered_float(m);
            L[j] = f;
            if (landmarks_next) landmarks_next[j] = f;
            Lmin[j] = 0xFFFFFFFFu;
        }
    } else if (landmarks_next) {
        for (int j = threadIdx.x; j < d; j += kT) landmarks_next[j] = L[j];
    }
    if (threadIdx.x == 0) *done3 = 0;
}

__global__ void k_iota(int32_t *a, uint32_t n) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = (int32_t)i;
}

__global__ void k_fill_u32(uint32_t *a, uint32_t n, uint32_t v) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_offsets(int64_t *off, int64_t T, int64_t N, int64_t n) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= T) off[t] = t < T ? t * N : n;
}

}  // namespace

subkm_status minmax_impl(subkm_ctx *ctx, const float *X, int64_t n, int32_t d, float *mins,
                         float *maxs, int *flag);

subkm_status subcluster_impl(subkm_ctx *ctx, const float *S, int64_t n, int32_t d, int64_t N,
                             int32_t landmark_mode, float *P, int32_t *perm, int64_t *offsets,
                             float *landmarks) {
    const int64_t T = ceil_div(n, N);
    hipStream_t s = ctx->stream;
    // scratch
    const uint32_t nb_max = (uint32_t)ceil_div(n, kBS);
    double *keys = (double *)ctx_scratch(ctx, SC_KEYS, sizeof(double) * n);
    int32_t *rem0 = (int32_t *)ctx_scratch(ctx, SC_REM0, sizeof(int32_t) * n);
    int32_t *rem1 = (int32_t *)ctx_scratch(ctx, SC_REM1, sizeof(int32_t) * n);
    char *cand = (char *)ctx_scratch(ctx, SC_CAND, (sizeof(double) + sizeof(uint32_t)) * n);
    const size_t sel_bytes = 256 + sizeof(uint32_t) * (2 * kBins + 2 * (size_t)nb_max + 64);
    char *sel = (char *)ctx_scratch(ctx, SC_SEL, sel_bytes);
    float *land = (float *)ctx_scratch(ctx, SC_LAND, sizeof(float) * 2 * d + 64);
    float *colmax = (float *)ctx_scratch(ctx, SC_COLMAX, sizeof(float) * d + 64);
    int *flag = (int *)ctx_scratch(ctx, SC_MM_FLAG, 256);
    if (!keys || !rem0 || !rem1 || !cand || !sel || !land || !colmax || !flag)
        return SUBKM_ENOMEM;
    SelState *st = (SelState *)sel;
    uint32_t *hist1 = (uint32_t *)(sel + 256);
    uint32_t *hist2 = hist1 + kBins;
    uint32_t *blockcnt = hist2 + kBins;
    uint32_t *blockoff = blockcnt + nb_max + 32;
    double *ckey = (double *)cand;
    uint32_t *cpos = (uint32_t *)(cand + sizeof(double) * n);
    float *L = land;
    uint32_t *Lmin = (uint32_t *)(land + d);

    SUBKM_HIP(ctx, hipMemsetAsync(sel, 0, sel_bytes, s));
    hipLaunchKernelGGL(k_fill_u32, dim3(ceil_div(d, 256)), dim3(256), 0, s, Lmin, (uint32_t)d,
                       0xFFFFFFFFu);
    SUBKM_LAUNCHED(ctx);
    // first landmark: attribute-wise minimum of all points; column maxima bound the keys
    SUBKM_TRY(minmax_impl(ctx, S, n, d, L, colmax, flag));
    hipLaunchKernelGGL(k_offsets, dim3(ceil_div(T + 1, 256)), dim3(256), 0, s, offsets, T, N, n);
    SUBKM_LAUNCHED(ctx);

    const bool fixed = landmark_mode == 1;
    const bool vec4 = (d % 4) == 0 && ((uintptr_t)S % 16) == 0;
    int32_t *cur = nullptr;  // round 0 uses the identity map
    int32_t *nxt = rem0;
    uint32_t nrem = (uint32_t)n;
    const size_t dyn_keys = sizeof(float) * d;
    const size_t dyn_scatter = sizeof(uint32_t) * d;
    for (int64_t t = 0; t < T; ++t) {
        const uint32_t need = (uint32_t)std::min<int64_t>(N, nrem);
        const uint32_t nb = (uint32_t)ceil_div(nrem, kBS);
        const bool all = need == nrem;
        float *lm_t = landmarks ? landmarks + t * d : nullptr;
        if (!all) {
            int64_t grid = std::min<int64_t>(ceil_div(nrem, kT), 512);
            if (!cur) {
                // round 0 reads the points in place; give k_keys an identity list
                hipLaunchKernelGGL(k_iota, dim3(ceil_div(nrem, 256)), dim3(256), 0, s, rem1, nrem);
                SUBKM_LAUNCHED(ctx);
                cur = rem1;
            }
            ProfScope pk(ctx, PK_KEYS);
            hipLaunchKernelGGL(k_keys, dim3(grid), dim3(kT), dyn_keys, s, S, d, cur, nrem, need, L,
                               colmax, keys, hist1, st, lm_t, vec4 ? 1 : 0);
            SUBKM_LAUNCHED(ctx);
            ProfScope pc(ctx, PK_CAND);
            hipLaunchKernelGGL(k_cand, dim3(nb), dim3(kT), 0, s, keys, nrem, need, st, ckey, cpos,
                               hist2, blockcnt, blockoff, nb);
            SUBKM_LAUNCHED(ctx);
        } else if (lm_t) {
            SUBKM_HIP(ctx, hipMemcpyAsync(lm_t, L, sizeof(float) * d, hipMemcpyDeviceToDevice, s));
        }
        const bool track = !all && !fixed;
        // L_{t+1} reaches `landmarks` through k_keys (or the copy above) of the next round
        float *lm_next = nullptr;
        ProfScope psc(ctx, PK_SCATTER);
        hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kT), dyn_scatter, s, S, d, cur, keys, nrem, st,
                           blockoff, all ? 1 : 0, track ? 1 : 0, P, perm, t * N, nxt, Lmin, L,
                           lm_next, &st->done3, need);
        SUBKM_LAUNCHED(ctx);
        nrem -= need;
        // the list just written becomes the current one
        int32_t *written = nxt;
        nxt = (written == rem0) ? rem1 : rem0;
        cur = written;
    }
    return SUBKM_OK;
}
