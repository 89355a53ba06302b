// Lloyd's k-means for many independent runs at once (Sec. II Algorithm 1
// step 4 inside every subcluster; Sec. I, Sec. V for the final run on the
// local centers).
//
// One iteration is two launches over all runs that are still active:
//
//   assign  work item = (run, tile of 256 points).  The run's centers are
//           staged in LDS; every thread keeps one point in registers and
//           tracks its two smallest float32 distances.  If their gap is not
//           larger than the rounding-error bound of the float32 arithmetic,
//           the point is re-assigned with binary64 distances, attributes left
//           to right, lowest center index on ties -- so every label is the
//           label of exact arithmetic on the float32 inputs.  The objective
//           of the tile (binary64 distance to the chosen center) goes to a
//           per-item slot.
//   update  work item = (run, chunk of centers).  The block scans the run's
//           labels, sums the points of its centers as 64-bit fixed point in
//           LDS (exact, so the result does not depend on the order of the
//           atomics), writes the new float32 centers (a center without
//           points stays) and its largest center move; the run's last block
//           decides convergence (largest move strictly below tol).
//
// A run's state moves ITER -> FINAL (converged: one more assignment gives
// labels and objective for the returned centers) -> DONE.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#pragma clang fp contract(off)

namespace {

constexpr int kAT = 256;        // assign threads = points per work item
constexpr int kUT = 256;        // update threads
constexpr int kLdsFloats = 8192;  // centers staged per assign pass (32 KB)
constexpr int kUpdLdsWords = 6144;  // int64 sums per update block (48 KB)

enum : int32_t { PH_ITER = 0, PH_FINAL = 1, PH_DONE = 2 };

struct DevRun {
    int64_t x_off, n, c_off, lab_off;
    int32_t d, k;
    int32_t item0, nitems;    // assign items
    int32_t uitem0, nuitems;  // update items
    int32_t kcu;              // centers per update item
    int32_t fix_shift;        // fixed-point exponent (set on the device)
};

struct RunState {
    int32_t phase;
    int32_t iters;
    uint32_t ucount;
    uint32_t pad;
    unsigned long long shift_bits;
    unsigned long long rechecks;
};

struct Item {
    int32_t run;
    int32_t first;  // first point (assign) or first center (update)
};

// ---------------------------------------------------------------------------
// exact binary64 distance of a float32 point to a float32 center, attributes
// left to right, separate multiply and add (the definition of the objective)
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
__device__ int32_t wave_argmin64(const float *x, const float *C, int d, int k, double *best_out) {
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
    *best_out = best;
    return bi;
}

// Deterministic sum of one double per thread (fixed pairing tree).
template <int NT>
__device__ double block_sum_det(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// Assignment.  D > 0: compile-time attribute count (point in registers);
// D == 0: any d (point read from global memory).
template <int D>
__global__ __launch_bounds__(kAT) void k_assign(const float *__restrict__ P,
                                                const DevRun *__restrict__ runs,
                                                const Item *__restrict__ items, int item_base,
                                                const float *__restrict__ C, int32_t *labels,
                                                RunState *rstate, double *ssepart) {
    __shared__ float sC[kLdsFloats];
    __shared__ int32_t s_list[kAT];
    __shared__ uint32_t s_nlist;
    __shared__ double s_red[kAT];
    __shared__ int32_t s_newlab[kAT];
    const Item it = items[item_base + blockIdx.x];
    const DevRun R = runs[it.run];
    if (rstate[it.run].phase == PH_DONE) return;
    const int d = D > 0 ? D : R.d;
    const int k = R.k;
    const int64_t i = it.first + threadIdx.x;
    const bool valid = i < R.n;
    const float *xg = P + R.x_off + (valid ? i : 0) * d;
    const float *Cr = C + R.c_off;
    float x[D > 0 ? D : 1];
    if (D > 0) {
#pragma unroll
        for (int j = 0; j < D; ++j) x[j] = valid ? xg[j] : 0.0f;
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
            // keep the two smallest; strict < keeps the lowest index first
            b2 = fminf(b2, fmaxf(acc, b1));
            bool lt = acc < b1;
            b1 = lt ? acc : b1;
            i1 = lt ? c0 + c : i1;
        }
    }
    // certain iff the gap exceeds the float32 error bound of both distances:
    // |D^ - D| <= gamma_{d+2} D (one rounding per subtraction, per FMA)
    const float gam = 2.0f * (float)(d + 2) * 5.9604645e-8f;
    const float slack = (float)(2 * d + 2) * 1.4012985e-45f * 2.0f;
    bool certain = (k == 1) || ((b2 - b1) > gam * (b1 + b2) + slack);
    if (valid && !certain) {
        uint32_t s = atomicAdd(&s_nlist, 1u);
        s_list[s] = threadIdx.x;
    }
    __syncthreads();
    // binary64 re-assignment of the uncertain points, one wavefront per point
    const uint32_t nl = s_nlist;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (uint32_t q = wave; q < nl; q += kAT / 64) {
        const int t = s_list[q];
        const float *xq = P + R.x_off + (it.first + t) * d;
        double bv;
        int32_t w = wave_argmin64(xq, Cr, d, k, &bv);
        if (lane == 0) s_newlab[t] = w;
    }
    __syncthreads();
    if (valid && !certain) i1 = s_newlab[threadIdx.x];
    double obj = 0.0;
    if (valid) {
        labels[R.lab_off + i] = i1;
        obj = dist64(xg, Cr + (int64_t)i1 * d, d);
    }
    double tot = block_sum_det<kAT>(obj, s_red);
    if (threadIdx.x == 0) {
        ssepart[item_base + blockIdx.x] = tot;
        if (nl) atomicAdd(&rstate[it.run].rechecks, (unsigned long long)nl);
    }
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ long long to_fixed(float x, int s) {
    return (long long)rint(ldexp((double)x, s));
}

// Update of one chunk of centers of one run.
__global__ __launch_bounds__(kUT) void k_update(const float *__restrict__ P,
                                                const DevRun *__restrict__ runs,
                                                const Item *__restrict__ items, int item_base,
                                                float *C, const int32_t *__restrict__ labels,
                                                RunState *rstate, double tol) {
    __shared__ long long s_sum[kUpdLdsWords];
    __shared__ unsigned int s_cnt[1024];
    __shared__ int32_t s_pts[kUT];
    __shared__ int32_t s_lab[kUT];
    __shared__ uint32_t s_np, s_last;
    __shared__ double s_red[kUT];
    const Item it = items[item_base + blockIdx.x];
    const DevRun R = runs[it.run];
    RunState *rs = rstate + it.run;
    const int32_t ph = rs->phase;
    if (ph == PH_DONE) return;
    if (ph == PH_FINAL) {
        // the assignment that just ran was the last one of this run
        if (it.first == 0 && threadIdx.x == 0) rs->phase = PH_DONE;
        return;
    }
    const int d = R.d;
    const int c0 = it.first;
    const int nc = R.kcu < R.k - c0 ? R.kcu : R.k - c0;
    const int s = R.fix_shift;
    for (int e = threadIdx.x; e < nc * d; e += kUT) s_sum[e] = 0;
    for (int c = threadIdx.x; c < nc; c += kUT) s_cnt[c] = 0;
    const float *X = P + R.x_off;
    const int32_t *lab = labels + R.lab_off;
    for (int64_t b = 0; b < R.n; b += kUT) {
        if (threadIdx.x == 0) s_np = 0;
        __syncthreads();
        int64_t i = b + threadIdx.x;
        if (i < R.n) {
            int32_t l = lab[i] - c0;
            if (l >= 0 && l < nc) {
                uint32_t q = atomicAdd(&s_np, 1u);
                s_pts[q] = (int32_t)threadIdx.x;
                s_lab[q] = l;
                atomicAdd(&s_cnt[l], 1u);
            }
        }
        __syncthreads();
        const int np = (int)s_np;
        for (int e = threadIdx.x; e < np * d; e += kUT) {
            int m = e / d, j = e - m * d;
            float v = X[(b + s_pts[m]) * d + j];
            atomicAdd((unsigned long long *)&s_sum[s_lab[m] * d + j],
                      (unsigned long long)to_fixed(v, s));
        }
        __syncthreads();
    }
    // new centers; squared moves go back into the sum slots as doubles
    float *Cr = C + R.c_off + (int64_t)c0 * d;
    for (int e = threadIdx.x; e < nc * d; e += kUT) {
        int c = e / d;
        unsigned int cnt = s_cnt[c];
        float old = Cr[e];
        double nv = cnt ? ldexp((double)s_sum[e], -s) / (double)cnt : (double)old;
        double mv = nv - (double)old;
        Cr[e] = (float)nv;
        s_sum[e] = __double_as_longlong(mv * mv);
    }
    __syncthreads();
    double mx = 0.0;
    for (int c = threadIdx.x; c < nc; c += kUT) {
        double a = 0.0;
        for (int j = 0; j < d; ++j) a = a + __longlong_as_double(s_sum[c * d + j]);
        mx = fmax(mx, sqrt(a));
    }
    // max over the block, then over the run (non-negative doubles order as
    // their bit patterns)
    s_red[threadIdx.x] = mx;
    __syncthreads();
    for (int st = kUT / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) s_red[threadIdx.x] = fmax(s_red[threadIdx.x], s_red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&rs->shift_bits, (unsigned long long)__double_as_longlong(s_red[0]));
        __threadfence();
        s_last = atomicAdd(&rs->ucount, 1u) == (uint32_t)R.nuitems - 1;
        if (s_last) {
            __threadfence();
            unsigned long long sb = __hip_atomic_load(&rs->shift_bits, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            double shift = __longlong_as_double((long long)sb);
            rs->iters += 1;
            rs->phase = shift < tol ? PH_FINAL : PH_ITER;
            rs->shift_bits = 0;
            rs->ucount = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// Per-run setup: fixed-point exponent from the largest |x| of the run, state.
__global__ __launch_bounds__(256) void k_setup(const float *__restrict__ P, DevRun *runs,
                                               RunState *rstate) {
    __shared__ float s_m[256];
    DevRun &R = runs[blockIdx.x];
    const float *X = P + R.x_off;
    const int64_t tot = R.n * R.d;
    float m = 0.0f;
    for (int64_t e = threadIdx.x; e < tot; e += 256) m = fmaxf(m, fabsf(X[e]));
    s_m[threadIdx.x] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) s_m[threadIdx.x] = fmaxf(s_m[threadIdx.x], s_m[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int e = 0;
        if (s_m[0] > 0.0f) frexpf(s_m[0], &e);  // max|x| < 2^e
        int lg = 0;
        while ((1ll << lg) < R.n + 1) ++lg;
        // n * 2^(e + s) <= 2^62 keeps every sum inside int64
        R.fix_shift = 61 - e - lg;
        RunState z{};
        z.phase = PH_ITER;
        rstate[blockIdx.x] = z;
    }
}

// first k points of every run as its starting centers (init 1), or the
// strided start C[q] = X[q * floor(n / k)] (init 2)
__global__ void k_init(const float *__restrict__ P, const DevRun *__restrict__ runs, float *C,
                       int mode) {
    const DevRun R = runs[blockIdx.y];
    const int64_t tot = (int64_t)R.k * R.d;
    const int64_t stride = mode == 2 ? R.n / R.k : 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t q = e / R.d, j = e - q * R.d;
        C[R.c_off + e] = P[R.x_off + q * stride * R.d + j];
    }
}

__global__ void k_finalize(const DevRun *__restrict__ runs, const RunState *__restrict__ rstate,
                           const double *__restrict__ ssepart, int R, int32_t *iters, double *sse) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const DevRun D = runs[r];
    double s = 0.0;
    for (int q = 0; q < D.nitems; ++q) s = s + ssepart[D.item0 + q];
    sse[r] = s;
    if (iters) iters[r] = rstate[r].iters;
}

template <int D>
subkm_status launch_assign(subkm_ctx *ctx, int nitems, int item_base, const float *P,
                           const DevRun *runs, const Item *items, const float *C, int32_t *labels,
                           RunState *rs, double *ssepart) {
    ProfScope ps(ctx, PK_ASSIGN);
    hipLaunchKernelGGL(k_assign<D>, dim3(nitems), dim3(kAT), 0, ctx->stream, P, runs, items,
                       item_base, C, labels, rs, ssepart);
    SUBKM_LAUNCHED(ctx);
    return SUBKM_OK;
}

subkm_status assign_dispatch(subkm_ctx *ctx, int d, int nitems, int item_base, const float *P,
                             const DevRun *runs, const Item *items, const float *C,
                             int32_t *labels, RunState *rs, double *ssepart) {
    if (nitems <= 0) return SUBKM_OK;
    switch (d) {
        case 1: return launch_assign<1>(ctx, nitems, item_base, P, runs, items, C, labels, rs, ssepart);
        case 2: return launch_assign<2>(ctx, nitems, item_base, P, runs, items, C, labels, rs, ssepart);
        case 4: return launch_assign<4>(ctx, nitems, item_base, P, runs, items, C, labels, rs, ssepart);
        case 8: return launch_assign<8>(ctx, nitems, item_base, P, runs, items, C, labels, rs, ssepart);
        case 16: return launch_assign<16>(ctx, nitems, item_base, P, runs, items, C, labels, rs, ssepart);
        case 32: return launch_assign<32>(ctx, nitems, item_base, P, runs, items, C, labels, rs, ssepart);
        case 64: return launch_assign<64>(ctx, nitems, item_base, P, runs, items, C, labels, rs, ssepart);
        case 128: return launch_assign<128>(ctx, nitems, item_base, P, runs, items, C, labels, rs, ssepart);
        default: return launch_assign<0>(ctx, nitems, item_base, P, runs, items, C, labels, rs, ssepart);
    }
}

}  // namespace

subkm_status lloyd_impl(subkm_ctx *ctx, const float *P, const subkm_run *runs, int32_t R,
                        float *C, int32_t *labels, int32_t max_iter, double tol,
                        int32_t precision, int32_t form, int32_t *iters, double *sse,
                        int init_mode) {
    (void)precision;
    hipStream_t s = ctx->stream;
    // host plan: order the assign items by attribute count so that one launch
    // covers all runs of one d; update items follow the run order
    std::vector<DevRun> dr(R);
    std::map<int, std::vector<int>> by_d;
    for (int r = 0; r < R; ++r) by_d[runs[r].d].push_back(r);
    std::vector<Item> items;
    std::vector<std::pair<int, std::pair<int, int>>> groups;  // d -> (item0, count)
    for (auto &g : by_d) {
        int g0 = (int)items.size();
        for (int r : g.second) {
            const subkm_run &u = runs[r];
            DevRun &D = dr[r];
            D.x_off = u.x_off;
            D.n = u.n;
            D.c_off = u.c_off;
            D.lab_off = u.lab_off;
            D.d = u.d;
            D.k = u.k;
            D.item0 = (int)items.size();
            for (int64_t f = 0; f < u.n; f += kAT) items.push_back(Item{r, (int32_t)f});
            D.nitems = (int)items.size() - D.item0;
        }
        groups.push_back({g.first, {g0, (int)items.size() - g0}});
    }
    const int n_assign = (int)items.size();
    for (int r = 0; r < R; ++r) {
        DevRun &D = dr[r];
        D.kcu = std::max(1, std::min({D.k, kUpdLdsWords / D.d, 1024}));
        D.uitem0 = (int)items.size();
        for (int c = 0; c < D.k; c += D.kcu) items.push_back(Item{r, c});
        D.nuitems = (int)items.size() - D.uitem0;
    }
    const int n_items = (int)items.size();
    const size_t b_runs = sizeof(DevRun) * R, b_items = sizeof(Item) * n_items;
    DevRun *d_runs = (DevRun *)ctx_scratch(ctx, SC_RUNS, b_runs + b_items);
    RunState *d_rs = (RunState *)ctx_scratch(ctx, SC_RSTATE, sizeof(RunState) * R);
    double *d_sse = (double *)ctx_scratch(ctx, SC_SSEPART, sizeof(double) * n_assign);
    char *h = (char *)ctx_pinned(ctx, b_runs + b_items);
    if (!d_runs || !d_rs || !d_sse || !h) return SUBKM_ENOMEM;
    Item *d_items = (Item *)((char *)d_runs + b_runs);
    // the pinned staging area is reused by the next call: wait for its copy
    SUBKM_HIP(ctx, hipStreamSynchronize(s));
    std::memcpy(h, dr.data(), b_runs);
    std::memcpy(h + b_runs, items.data(), b_items);
    SUBKM_HIP(ctx, hipMemcpyAsync(d_runs, h, b_runs + b_items, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_setup, dim3(R), dim3(256), 0, s, P, d_runs, d_rs);
    SUBKM_LAUNCHED(ctx);
    if (init_mode) {
        int64_t kmax = 0;
        for (int r = 0; r < R; ++r) kmax = std::max<int64_t>(kmax, (int64_t)runs[r].k * runs[r].d);
        hipLaunchKernelGGL(k_init, dim3(std::min<int64_t>(ceil_div(kmax, 256), 1024), R), dim3(256),
                           0, s, P, d_runs, C, init_mode);
        SUBKM_LAUNCHED(ctx);
    }
    if (form == SUBKM_FORM_PLAIN) {
        // one run at a time, one launch per phase
        for (int r = 0; r < R; ++r) {
            const DevRun &D = dr[r];
            for (int a = 0; a <= max_iter; ++a) {
                SUBKM_TRY(assign_dispatch(ctx, D.d, D.nitems, D.item0, P, d_runs, d_items, C,
                                          labels, d_rs, d_sse));
                if (a < max_iter) {
                    ProfScope ps(ctx, PK_UPDATE);
                    hipLaunchKernelGGL(k_update, dim3(D.nuitems), dim3(kUT), 0, s, P, d_runs,
                                       d_items, D.uitem0, C, labels, d_rs, tol);
                    SUBKM_LAUNCHED(ctx);
                }
            }
        }
    } else {
        const int u0 = n_assign, nu = n_items - n_assign;
        for (int a = 0; a <= max_iter; ++a) {
            for (auto &g : groups)
                SUBKM_TRY(assign_dispatch(ctx, g.first, g.second.second, g.second.first, P,
                                          d_runs, d_items, C, labels, d_rs, d_sse));
            if (a < max_iter) {
                ProfScope ps(ctx, PK_UPDATE);
                hipLaunchKernelGGL(k_update, dim3(nu), dim3(kUT), 0, s, P, d_runs, d_items, u0, C,
                                   labels, d_rs, tol);
                SUBKM_LAUNCHED(ctx);
            }
        }
    }
    hipLaunchKernelGGL(k_finalize, dim3(ceil_div(R, 256)), dim3(256), 0, s, d_runs, d_rs, d_sse, R,
                       iters, sse);
    SUBKM_LAUNCHED(ctx);
    return SUBKM_OK;
}
