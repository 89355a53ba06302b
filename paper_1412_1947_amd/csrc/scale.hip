// Min-max feature scaling (Sec. II, Algorithm 1 step 1; Sec. III, Algorithm 2
// step 1).  Two HBM-bound passes: column minima/maxima (exact, so the
// reduction order is free), then the binary64 transform rounded once to
// float32.
//
// Thread -> element mapping.  Narrow rows (d < 64): a flat grid-stride loop
// whose stride is a multiple of d, so every thread keeps one fixed column and
// consecutive lanes read consecutive floats.  Wide rows (d >= 64): a block
// owns a range of rows; its threads split into row groups whose lanes cover
// the (float4) columns of a row, contiguous across lanes, each walking its
// group's rows with several rows in flight.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <numeric>

#pragma clang fp contract(off)

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_minmax_narrow(const float *__restrict__ X,
                                                            int64_t total, int d, int64_t stride,
                                                            float *__restrict__ pmin,
                                                            float *__restrict__ pmax,
                                                            int *__restrict__ flag) {
    __shared__ float smin[kThreads], smax[kThreads];
    const int t = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * kThreads + t;
    float mn = INFINITY, mx = -INFINITY;
    bool bad = false;
    for (int64_t e = e0; e < total; e += stride) {
        float v = __builtin_nontemporal_load(X + e);
        bad |= !isfinite(v);
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
    }
    if (bad) atomicOr(flag, 1);
    smin[t] = mn;
    smax[t] = mx;
    __syncthreads();
    // column c collects the threads t' with (blockIdx*256 + t') % d == c
    const int base = (int)(((int64_t)blockIdx.x * kThreads) % d);
    for (int c = t; c < d; c += kThreads) {
        int t0 = (c - base) % d;
        if (t0 < 0) t0 += d;
        float a = INFINITY, b = -INFINITY;
        for (int q = t0; q < kThreads; q += d) {
            a = fminf(a, smin[q]);
            b = fmaxf(b, smax[q]);
        }
        pmin[(int64_t)blockIdx.x * d + c] = a;
        pmax[(int64_t)blockIdx.x * d + c] = b;
    }
}

// Wide rows: a block owns rows [r0, r1).  Its threads form row groups of
// `span` threads, one thread per W-float column vector (a block handles up
// to kThreads vectors of a row at a time); each thread walks its group's
// rows with kRU rows in flight, and the row groups meet in LDS.
template <int W>
struct VecW;
template <>
struct VecW<1> {
    using T = float;
    static __device__ __forceinline__ float get(const float &v, int) { return v; }
    static __device__ __forceinline__ void set(float &v, int, float x) { v = x; }
};
template <>
struct VecW<4> {
    using T = float4;
    static __device__ __forceinline__ float get(const float4 &v, int c) {
        return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w;
    }
    static __device__ __forceinline__ void set(float4 &v, int c, float x) {
        if (c == 0) v.x = x;
        else if (c == 1) v.y = x;
        else if (c == 2) v.z = x;
        else v.w = x;
    }
};

constexpr int kRU = 4;  // rows in flight per thread

template <int W>
__global__ __launch_bounds__(kThreads) void k_minmax_wide(const float *__restrict__ X, int64_t n,
                                                          int d, int64_t rows_per_block,
                                                          float *__restrict__ pmin,
                                                          float *__restrict__ pmax,
                                                          int *__restrict__ flag) {
    using V = typename VecW<W>::T;
    __shared__ float smn[kThreads * W], smx[kThreads * W];
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    const int dv = d / W;
    const V *Xv = (const V *)X;
    bool bad = false;
    for (int cb = 0; cb < dv; cb += kThreads) {
        const int span = min(kThreads, dv - cb);
        const int rp = kThreads / span;
        const int rg = threadIdx.x / span, cv = cb + threadIdx.x % span;
        float mn[W], mx[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            mn[w] = INFINITY;
            mx[w] = -INFINITY;
        }
        if (rg < rp) {
            int64_t r = r0 + rg;
            for (; r + (int64_t)(kRU - 1) * rp < r1; r += (int64_t)kRU * rp) {
                V v[kRU];
#pragma unroll
                for (int u = 0; u < kRU; ++u) v[u] = Xv[(r + (int64_t)u * rp) * dv + cv];
#pragma unroll
                for (int u = 0; u < kRU; ++u)
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const float x = VecW<W>::get(v[u], w);
                        bad |= !isfinite(x);
                        mn[w] = fminf(mn[w], x);
                        mx[w] = fmaxf(mx[w], x);
                    }
            }
            for (; r < r1; r += rp) {
                const V v = Xv[r * dv + cv];
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const float x = VecW<W>::get(v, w);
                    bad |= !isfinite(x);
                    mn[w] = fminf(mn[w], x);
                    mx[w] = fmaxf(mx[w], x);
                }
            }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
            smn[threadIdx.x * W + w] = mn[w];
            smx[threadIdx.x * W + w] = mx[w];
        }
        __syncthreads();
        if ((int)threadIdx.x < span) {
            for (int g = 1; g < rp; ++g)
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    mn[w] = fminf(mn[w], smn[(g * span + threadIdx.x) * W + w]);
                    mx[w] = fmaxf(mx[w], smx[(g * span + threadIdx.x) * W + w]);
                }
#pragma unroll
            for (int w = 0; w < W; ++w) {
                pmin[(int64_t)blockIdx.x * d + cv * W + w] = mn[w];
                pmax[(int64_t)blockIdx.x * d + cv * W + w] = mx[w];
            }
        }
        __syncthreads();
    }
    if (bad) atomicOr(flag, 1);
}

// second stage: one block per column, a strided pass over the block
// partials and a tree in LDS (min and max are exact in any order)
__global__ __launch_bounds__(256) void k_minmax_final(const float *__restrict__ pmin,
                                                      const float *__restrict__ pmax, int parts,
                                                      int d, float *__restrict__ mins,
                                                      float *__restrict__ maxs) {
    __shared__ float sa[256], sb[256];
    const int c = blockIdx.x;
    float a = INFINITY, b = -INFINITY;
    for (int p = threadIdx.x; p < parts; p += 256) {
        a = fminf(a, pmin[(int64_t)p * d + c]);
        b = fmaxf(b, pmax[(int64_t)p * d + c]);
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sa[threadIdx.x] = fminf(sa[threadIdx.x], sa[threadIdx.x + s]);
            sb[threadIdx.x] = fmaxf(sb[threadIdx.x], sb[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (mins) mins[c] = sa[0];
        if (maxs) maxs[c] = sb[0];
    }
}

__device__ __forceinline__ float scale_one(float x, float mn, float mx) {
    double range = (double)mx - (double)mn;
    if (!(range > 0.0)) return 0.0f;
    double num = (double)x - (double)mn;
    return (float)(num / range);
}

__global__ __launch_bounds__(kThreads) void k_apply_narrow(const float *X, int64_t total, int d,
                                                           int64_t stride,
                                                           const float *__restrict__ mins,
                                                           const float *__restrict__ maxs,
                                                           float *S) {
    const int64_t e0 = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e0 >= total) return;
    const int c = (int)(e0 % d);
    const float mn = mins[c], mx = maxs[c];
    for (int64_t e = e0; e < total; e += stride) S[e] = scale_one(X[e], mn, mx);
}

template <int W>
__global__ __launch_bounds__(kThreads) void k_apply_wide(const float *X, int64_t n, int d,
                                                         int64_t rows_per_block,
                                                         const float *__restrict__ mins,
                                                         const float *__restrict__ maxs,
                                                         float *S) {
    using V = typename VecW<W>::T;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    const int dv = d / W;
    const V *Xv = (const V *)X;
    V *Sv = (V *)S;
    for (int cb = 0; cb < dv; cb += kThreads) {
        const int span = min(kThreads, dv - cb);
        const int rp = kThreads / span;
        const int rg = threadIdx.x / span, cv = cb + threadIdx.x % span;
        if (rg >= rp) continue;
        float mn[W], mx[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            mn[w] = mins[cv * W + w];
            mx[w] = maxs[cv * W + w];
        }
        int64_t r = r0 + rg;
        for (; r + (int64_t)(kRU - 1) * rp < r1; r += (int64_t)kRU * rp) {
            V v[kRU];
#pragma unroll
            for (int u = 0; u < kRU; ++u) v[u] = Xv[(r + (int64_t)u * rp) * dv + cv];
#pragma unroll
            for (int u = 0; u < kRU; ++u) {
                V o;
#pragma unroll
                for (int w = 0; w < W; ++w) VecW<W>::set(o, w, scale_one(VecW<W>::get(v[u], w), mn[w], mx[w]));
                Sv[(r + (int64_t)u * rp) * dv + cv] = o;
            }
        }
        for (; r < r1; r += rp) {
            const V v = Xv[r * dv + cv];
            V o;
#pragma unroll
            for (int w = 0; w < W; ++w) VecW<W>::set(o, w, scale_one(VecW<W>::get(v, w), mn[w], mx[w]));
            Sv[r * dv + cv] = o;
        }
    }
}

// Column-major input (attribute j of point i at X[j n + i], the paper's
// column-major flattening).  Minima/maxima: block (chunk, column) reduces a
// contiguous stretch of one column with float4 loads; the partials use the
// row-major layout of k_minmax_final.
constexpr int kCmChunk = 16384;  // points per partial

__global__ __launch_bounds__(kThreads) void k_minmax_cm(const float *__restrict__ X, int64_t n,
                                                        int d, int vec4,
                                                        float *__restrict__ pmin,
                                                        float *__restrict__ pmax,
                                                        int *__restrict__ flag) {
    __shared__ float sa[kThreads], sb[kThreads];
    const int j = blockIdx.y;
    const int64_t i0 = (int64_t)blockIdx.x * kCmChunk;
    const int64_t i1 = min(n, i0 + kCmChunk);
    const float *col = X + (int64_t)j * n;
    float mn = INFINITY, mx = -INFINITY;
    bool bad = false;
    auto take = [&](float x) {
        bad |= !isfinite(x);
        mn = fminf(mn, x);
        mx = fmaxf(mx, x);
    };
    if (vec4) {
        const float4 *c4 = (const float4 *)(col + i0);
        const int64_t nv = (i1 - i0) >> 2;
        for (int64_t v = threadIdx.x; v < nv; v += kThreads) {
            const float4 q = c4[v];
            take(q.x);
            take(q.y);
            take(q.z);
            take(q.w);
        }
        for (int64_t i = i0 + 4 * nv + threadIdx.x; i < i1; i += kThreads) take(col[i]);
    } else {
        for (int64_t i = i0 + threadIdx.x; i < i1; i += kThreads) take(col[i]);
    }
    sa[threadIdx.x] = mn;
    sb[threadIdx.x] = mx;
    __syncthreads();
    for (int st = kThreads / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sa[threadIdx.x] = fminf(sa[threadIdx.x], sa[threadIdx.x + st]);
            sb[threadIdx.x] = fmaxf(sb[threadIdx.x], sb[threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pmin[(int64_t)blockIdx.x * d + j] = sa[0];
        pmax[(int64_t)blockIdx.x * d + j] = sb[0];
    }
    if (bad) atomicOr(flag, 1);
}

// Scaling with the transpose to row-major S: a block moves a tile of 64
// points x 64 attributes through LDS, reading along points (contiguous in X)
// and writing along attributes (contiguous in S).
__global__ __launch_bounds__(kThreads) void k_apply_cm(const float *__restrict__ X, int64_t n, int d,
                                                       const float *__restrict__ mins,
                                                       const float *__restrict__ maxs,
                                                       float *__restrict__ S) {
    __shared__ float tile[64][65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int j0 = blockIdx.y * 64;
    const int ti = threadIdx.x & 63, tq = threadIdx.x >> 6;
    for (int jj = tq; jj < 64; jj += kThreads / 64) {
        const int j = j0 + jj;
        const int64_t i = i0 + ti;
        tile[jj][ti] = (j < d && i < n) ? X[(int64_t)j * n + i] : 0.0f;
    }
    __syncthreads();
    for (int ii = tq; ii < 64; ii += kThreads / 64) {
        const int64_t i = i0 + ii;
        const int j = j0 + ti;
        if (i < n && j < d) S[i * d + j] = scale_one(tile[ti][ii], mins[j], maxs[j]);
    }
}

struct Plan {
    bool narrow;
    int64_t blocks;
    int64_t stride;          // narrow: elements
    int64_t rows_per_block;  // wide
};

// max_blocks caps the wide form's grid (its partials take 2 d floats per
// block); the narrow form has at most 2048 + 62 blocks.
Plan plan_for(int64_t n, int d, int64_t max_blocks = 2048) {
    Plan p{};
    const int64_t total = n * d;
    if (d < 64) {
        p.narrow = true;
        const int64_t unit = d / std::gcd(d, kThreads);  // blocks per column period
        int64_t want = std::min<int64_t>(ceil_div(total, kThreads), 2048);
        p.blocks = std::max<int64_t>(unit, ceil_div(want, unit) * unit);
        p.stride = p.blocks * kThreads;
    } else {
        p.narrow = false;
        p.rows_per_block = std::max<int64_t>(8, ceil_div(n, std::min<int64_t>(2048, max_blocks)));
        p.blocks = ceil_div(n, p.rows_per_block);
    }
    return p;
}

// Column minima/maxima (partials into pmin/pmax, then the final reduction)
// and the transform, for a plan; shared by the entry points that take their
// partials from the context's scratch and from the static scratch below.
void launch_minmax(hipStream_t s, const Plan &p, const float *X, int64_t n, int d, float *pmin,
                   float *pmax, int *flag, float *mins, float *maxs) {
    if (p.narrow)
        hipLaunchKernelGGL(k_minmax_narrow, dim3(p.blocks), dim3(kThreads), 0, s, X, n * d, d,
                           p.stride, pmin, pmax, flag);
    else if (d % 4 == 0 && (uintptr_t)X % 16 == 0)
        hipLaunchKernelGGL(k_minmax_wide<4>, dim3(p.blocks), dim3(kThreads), 0, s, X, n, d,
                           p.rows_per_block, pmin, pmax, flag);
    else
        hipLaunchKernelGGL(k_minmax_wide<1>, dim3(p.blocks), dim3(kThreads), 0, s, X, n, d,
                           p.rows_per_block, pmin, pmax, flag);
    hipLaunchKernelGGL(k_minmax_final, dim3(d), dim3(256), 0, s, pmin, pmax, (int)p.blocks, d, mins,
                       maxs);
}

void launch_apply(hipStream_t s, const Plan &p, const float *X, int64_t n, int d,
                  const float *mins, const float *maxs, float *S) {
    if (p.narrow)
        hipLaunchKernelGGL(k_apply_narrow, dim3(p.blocks), dim3(kThreads), 0, s, X, n * d, d,
                           p.stride, mins, maxs, S);
    else if (d % 4 == 0 && (uintptr_t)X % 16 == 0 && (uintptr_t)S % 16 == 0)
        hipLaunchKernelGGL(k_apply_wide<4>, dim3(p.blocks), dim3(kThreads), 0, s, X, n, d,
                           p.rows_per_block, mins, maxs, S);
    else
        hipLaunchKernelGGL(k_apply_wide<1>, dim3(p.blocks), dim3(kThreads), 0, s, X, n, d,
                           p.rows_per_block, mins, maxs, S);
}

__global__ void k_clear_word(int *w) { *w = 0; }

}  // namespace

size_t minmax_cm_scratch_bytes(int64_t n, int32_t d) {
    return sizeof(float) * 2 * (size_t)ceil_div(n, kCmChunk) * d;
}

// Scaling of a column-major X into row-major S (Sec. V's column-major
// flattening as an input layout); the same arithmetic as scale_impl.
subkm_status scale_cm_impl(subkm_ctx *ctx, const float *X, int64_t n, int32_t d, float *S,
                           float *mins, float *maxs, bool check_finite) {
    int *flag = (int *)ctx_scratch(ctx, SC_MM_FLAG, 256);
    if (!flag) return SUBKM_ENOMEM;
    SUBKM_HIP(ctx, hipMemsetAsync(flag, 0, sizeof(int), ctx->stream));
    const int64_t parts = ceil_div(n, kCmChunk);
    float *part = (float *)ctx_scratch(ctx, SC_MM_PART, minmax_cm_scratch_bytes(n, d));
    if (!part) return SUBKM_ENOMEM;
    float *pmin = part, *pmax = part + parts * d;
    {
        ProfScope ps(ctx, PK_SCALE);
        const int vec4 = ((uintptr_t)X % 16 == 0 && n % 4 == 0) ? 1 : 0;
        hipLaunchKernelGGL(k_minmax_cm, dim3((unsigned)parts, (unsigned)d), dim3(kThreads), 0,
                           ctx->stream, X, n, d, vec4, pmin, pmax, flag);
        SUBKM_LAUNCHED(ctx);
        hipLaunchKernelGGL(k_minmax_final, dim3(d), dim3(256), 0, ctx->stream, pmin, pmax,
                           (int)parts, d, mins, maxs);
        SUBKM_LAUNCHED(ctx);
    }
    if (check_finite) {
        int *h = (int *)ctx_pinned(ctx, sizeof(int));
        if (!h) return SUBKM_ENOMEM;
        SUBKM_HIP(ctx, hipMemcpyAsync(h, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        SUBKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (*h) return set_err(ctx, SUBKM_EINVAL, "input contains NaN or infinite values");
    }
    ProfScope ps(ctx, PK_SCALE);
    hipLaunchKernelGGL(k_apply_cm, dim3((unsigned)ceil_div(n, 64), (unsigned)ceil_div(d, 64)),
                       dim3(kThreads), 0, ctx->stream, X, n, d, mins, maxs, S);
    SUBKM_LAUNCHED(ctx);
    return SUBKM_OK;
}

// scratch bytes minmax_impl asks for (callers that capture graphs allocate first)
size_t minmax_scratch_bytes(int64_t n, int32_t d) {
    Plan p = plan_for(n, d);
    return sizeof(float) * 2 * p.blocks * d;
}

// Column minima and maxima of an n x d array into mins/maxs (either may be
// null).  flag (device int, zeroed by the caller) is set when a value is NaN
// or infinite.
subkm_status minmax_impl(subkm_ctx *ctx, const float *X, int64_t n, int32_t d, float *mins,
                         float *maxs, int *flag) {
    ProfScope ps(ctx, PK_SCALE);
    Plan p = plan_for(n, d);
    float *part = (float *)ctx_scratch(ctx, SC_MM_PART, sizeof(float) * 2 * p.blocks * d);
    if (!part) return SUBKM_ENOMEM;
    launch_minmax(ctx->stream, p, X, n, d, part, part + p.blocks * d, flag, mins, maxs);
    SUBKM_LAUNCHED(ctx);
    return SUBKM_OK;
}

subkm_status scale_impl(subkm_ctx *ctx, const float *X, int64_t n, int32_t d, float *S,
                        float *mins, float *maxs, bool check_finite) {
    int *flag = (int *)ctx_scratch(ctx, SC_MM_FLAG, 256);
    if (!flag) return SUBKM_ENOMEM;
    SUBKM_HIP(ctx, hipMemsetAsync(flag, 0, sizeof(int), ctx->stream));
    SUBKM_TRY(minmax_impl(ctx, X, n, d, mins, maxs, flag));
    if (check_finite) {
        int *h = (int *)ctx_pinned(ctx, sizeof(int));
        if (!h) return SUBKM_ENOMEM;
        SUBKM_HIP(ctx, hipMemcpyAsync(h, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        SUBKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (*h) return set_err(ctx, SUBKM_EINVAL, "input contains NaN or infinite values");
    }
    ProfScope ps(ctx, PK_SCALE);
    launch_apply(ctx->stream, plan_for(n, d), X, n, d, mins, maxs, S);
    SUBKM_LAUNCHED(ctx);
    return SUBKM_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free scaling (subkm_scale_noalloc).  Its scratch -- the
// non-finite flag in the first 256 bytes, then the min/max partials -- is
// this file-scope device array, which every GPU the library runs on holds
// once, at its own address, until the process ends.  In host code the
// array's name is not a device address: the address is looked up per
// device with hipGetSymbolAddress when a context is created, and only that
// address is handed to kernels.
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
constexpr size_t kNoAllocFlagBytes = 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kNoAllocDevices] = {};
hipError_t g_noalloc_err[kNoAllocDevices] = {};
bool g_noalloc_done[kNoAllocDevices] = {};
}  // namespace

void noalloc_scratch_init(subkm_ctx *ctx) {
    // the caller has made ctx->device current
    const int dev = ctx->device;
    ctx->noalloc_scratch = nullptr;
    if (dev < 0 || dev >= kNoAllocDevices) return;
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    if (!g_noalloc_done[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            hipGetLastError();
            p = nullptr;
        }
        g_noalloc_ptr[dev] = p;
        g_noalloc_err[dev] = e;
        g_noalloc_done[dev] = true;
    }
    ctx->noalloc_scratch = g_noalloc_ptr[dev];
    ctx->noalloc_err = g_noalloc_err[dev];
}

subkm_status scale_noalloc_impl(subkm_ctx *ctx, const float *X, int64_t n, int32_t d, float *S,
                                float *mins, float *maxs) {
    if (!ctx->noalloc_scratch)
        return set_err(ctx, SUBKM_EDEVICE, "the static scratch of device %d has no address: %s",
                       ctx->device, hipGetErrorString(ctx->noalloc_err));
    // the wide form's grid is capped so that its partials fit; the narrow
    // form needs at most 2 * 2110 * 63 floats
    const int64_t cap = (int64_t)((kNoAllocScratchBytes - kNoAllocFlagBytes) / (2 * sizeof(float) * d));
    const Plan p = plan_for(n, d, std::max<int64_t>(1, cap));
    const size_t need = kNoAllocFlagBytes + sizeof(float) * 2 * (size_t)p.blocks * d;
    if (need > kNoAllocScratchBytes)
        return set_err(ctx, SUBKM_EINVAL, "n = %lld, d = %d needs %zu bytes of scratch; the static "
                       "scratch holds %zu", (long long)n, d, need, kNoAllocScratchBytes);
    hipStream_t s = ctx->stream;
    int *flag = (int *)ctx->noalloc_scratch;
    float *part = (float *)((unsigned char *)ctx->noalloc_scratch + kNoAllocFlagBytes);
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(1), 0, s, flag);
    SUBKM_LAUNCHED(ctx);
    launch_minmax(s, p, X, n, d, part, part + p.blocks * d, flag, mins, maxs);
    SUBKM_LAUNCHED(ctx);
    int h = 0;
    SUBKM_HIP(ctx, hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    SUBKM_HIP(ctx, hipStreamSynchronize(s));
    if (h) return set_err(ctx, SUBKM_EINVAL, "input contains NaN or infinite values");
    launch_apply(s, p, X, n, d, mins, maxs, S);
    SUBKM_LAUNCHED(ctx);
    return SUBKM_OK;
}
