// Internal declarations of libsubkm (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/subkm.h"

// ---------------------------------------------------------------------------
// Context: device, stream, scratch slots that persist between calls.
enum ScratchSlot {
    SC_MM_PART = 0,  // min/max partials
    SC_MM_FLAG,      // non-finite flag + small host-visible words
    SC_KEYS,         // landmark keys, double per remaining point
    SC_REM0,         // remaining positions -> original index (ping)
    SC_REM1,         // (pong)
    SC_CAND,         // selection candidates (key, position)
    SC_SEL,          // selection state + histograms + block counts
    SC_LAND,         // landmark (float), running minima (ordered uint), minimum-holder keys
    SC_COLMAX,       // column maxima of S for the key bound
    SC_RUNS,         // device copy of run descriptors
    SC_ITEMS,        // work items of the Lloyd kernels
    SC_RSTATE,       // per-run Lloyd state
    SC_SSEPART,      // per-item objective partials
    SC_FIXSCALE,     // per-run fixed-point exponents
    SC_RECHECK,      // recheck counters
    SC_CL_S,         // cluster(): scaled points
    SC_CL_P,         // cluster(): grouped points
    SC_CL_PERM,      // cluster(): permutation
    SC_CL_OFFS,      // cluster(): offsets
    SC_CL_LOCAL,     // cluster(): local centers
    SC_CL_LLAB,      // cluster(): local labels
    SC_CL_LIT,       // cluster(): local iterations
    SC_CL_LSSE,      // cluster(): local objective
    SC_CL_MINMAX,    // cluster(): mins / maxs
    SC_CL_FINAL,     // cluster(): final-run labels, iters, sse
    SC_BOX,          // per-run attribute bounds
    SC_WCNT,         // wide runs: counts | starts | cursors per center
    SC_WORDER,       // wide runs: point indices grouped by label
    SC_FRAGS,        // split path: center fragments
    SC_CNORM,        // split path: squared center norms
    SC_UQ,           // unequal subclustering: bounds, landmark basis, histograms
    SC_UQ_GROUP,     // unequal subclustering: group of every point
    SC_UQ_LOCAL,     // cluster() with unequal groups: run -> group map, local outputs
    SC_TUNE,         // schedule tuner: the caller's starting centers
    SC_COUNT
};

// Kernel classes timed by the optional per-launch profiler (device events on
// the context's stream around every launch of the class).
enum ProfClass {
    PK_ASSIGN = 0, PK_UPDATE, PK_KEYS, PK_CAND, PK_SCATTER, PK_SCALE, PK_LLOYD_FUSED,
    PK_SUBCLUSTER, PK_COUNT
};

struct ProfRec {
    int cls;
    hipEvent_t a, b;
};

// Contexts that share a device inside one serving engine run their
// cooperative (persistent) launches one after the other: each such launch
// waits on the GPU for the previous one, so two grids never hold parts of
// the device while they wait for their own missing blocks.
struct CoopGate {
    std::mutex mu;
    hipEvent_t ev = nullptr;
    bool armed = false;
};

// Schedule of the batched Lloyd form (results do not depend on it): the
// largest number of blocks per run, the divisor of the co-resident grid,
// the fewest 256-point tiles a block of a split run takes per move, and how
// the blocks of a run combine their sums every move (0: every block
// publishes its part, then each sums a slice of the parts, two arrivals;
// 1: every block adds its part into shared totals, one arrival).
struct LloydSched {
    int32_t gcap;
    int32_t bdiv;
    int32_t tpb;
    int32_t xmode;
};
struct TuneKey {
    uint64_t v[5];
    bool operator<(const TuneKey &o) const {
        for (int i = 0; i < 5; ++i)
            if (v[i] != o.v[i]) return v[i] < o.v[i];
        return false;
    }
};
struct TuneEntry {
    LloydSched sched;
    double ms;
};

struct ScratchBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct subkm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int cu_count = 256;
    std::string err;
    ScratchBuf scratch[SC_COUNT];
    void *pinned = nullptr;  // small pinned host area (flags read back after a sync)
    size_t pinned_bytes = 0;
    // Pinned staging of the Lloyd plans, a ring: a call writes its plan into
    // the next slot and records an event after the slot's host-to-device
    // copy, so it waits (rarely) only for the copy issued kStageSlots calls
    // earlier, never for the stream to drain.
    static constexpr int kStageSlots = 4;
    struct Stage {
        void *h = nullptr;
        size_t bytes = 0;
        hipEvent_t ev = nullptr;
        bool pending = false;
    };
    Stage stage[kStageSlots];
    int stage_next = 0;
    // Sticky device flags (zeroed at creation): word 0 is set by a
    // persistent Lloyd launch whose barrier gave up; subkm_synchronize
    // reports and clears it.
    int *sticky = nullptr;
    // device address of the static scratch of subkm_scale_noalloc on this
    // context's device (nullptr when the lookup failed, with its error)
    void *noalloc_scratch = nullptr;
    hipError_t noalloc_err = hipSuccess;
    hipEvent_t ev[8] = {};
    bool prof_on = false;
    std::vector<ProfRec> prof_pending;
    std::vector<hipEvent_t> prof_free;
    double prof_ms[PK_COUNT] = {};
    long long prof_n[PK_COUNT] = {};
    uint64_t scratch_epoch = 0;       // bumped whenever a scratch buffer moves
    hipStream_t cap_stream = nullptr;  // private stream for graph capture
    CoopGate *coop = nullptr;          // serving engine: shared gate of cooperative launches
    static constexpr int kGraphKeyWords = 21;
    static constexpr size_t kGraphCacheMax = 8;
    struct GraphCache {
        bool valid = false;
        uint64_t key[kGraphKeyWords] = {};
        uint64_t stamp = 0;            // last use (least recently used is replaced)
        hipGraphExec_t exec = nullptr;
    };
    std::vector<GraphCache> subg;      // captured subclustering sequences
    uint64_t subg_clock = 0;
    bool tune_on = false;              // tune the schedules of unseen shapes
    std::map<TuneKey, TuneEntry> tune; // tuned schedule per shape
};

// RAII timer of the launches issued inside its scope (no-op when off).
struct ProfScope {
    subkm_ctx *ctx;
    int cls;
    hipEvent_t a = nullptr;
    ProfScope(subkm_ctx *c, int k);
    ~ProfScope();
};

// Scratch memory of a slot with at least `bytes` bytes (grows on demand).
// Returns nullptr and sets ctx->err when allocation fails.
void *ctx_scratch(subkm_ctx *ctx, int slot, size_t bytes);
void *ctx_pinned(subkm_ctx *ctx, size_t bytes);
// Next slot of the plan staging ring with at least `bytes` bytes; *slot
// receives its index for ctx_stage_issued (nullptr and ctx->err on failure).
void *ctx_stage(subkm_ctx *ctx, size_t bytes, int *slot);
// The copy out of staging slot `slot` has been issued on the context's stream.
subkm_status ctx_stage_issued(subkm_ctx *ctx, int slot);

subkm_status set_err(subkm_ctx *ctx, subkm_status st, const char *fmt, ...);

#define SUBKM_HIP(ctx, expr)                                                              \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return set_err((ctx), SUBKM_EDEVICE, "%s failed: %s (%s:%d)", #expr,          \
                           hipGetErrorString(e_), __FILE__, __LINE__);                    \
    } while (0)

#define SUBKM_LAUNCHED(ctx)                                                               \
    do {                                                                                  \
        hipError_t e_ = hipGetLastError();                                                \
        if (e_ != hipSuccess)                                                             \
            return set_err((ctx), SUBKM_EDEVICE, "kernel launch failed: %s (%s:%d)",      \
                           hipGetErrorString(e_), __FILE__, __LINE__);                    \
    } while (0)

#define SUBKM_TRY(expr)                                                                   \
    do {                                                                                  \
        subkm_status s_ = (expr);                                                         \
        if (s_ != SUBKM_OK) return s_;                                                    \
    } while (0)

// ---------------------------------------------------------------------------
// Stage entry points used by subkm_cluster (already validated arguments).
subkm_status scale_impl(subkm_ctx *ctx, const float *X, int64_t n, int32_t d, float *S,
                        float *mins, float *maxs, bool check_finite);
// The same for a column-major X (X[j n + i]); S is row-major.
subkm_status scale_cm_impl(subkm_ctx *ctx, const float *X, int64_t n, int32_t d, float *S,
                           float *mins, float *maxs, bool check_finite);
subkm_status subcluster_impl(subkm_ctx *ctx, const float *S, int64_t n, int32_t d, int64_t N,
                             int32_t landmark_mode, int32_t metric, float *P, int32_t *perm,
                             int64_t *offsets, float *landmarks);
subkm_status subcluster_selections(subkm_ctx *ctx, const float *S, const float *P, int64_t n,
                                   int32_t d, int64_t N, int32_t metric, int64_t *out);
// Largest number of groups of the unequal subclustering (one LDS counter per
// group in the histogram and placement kernels).
constexpr int64_t kUqMaxGroups = 8192;
// Unequal sized subclustering (Algorithm 2) into m groups: P, perm (n),
// offsets (m + 1), landmarks (nullable, m x d binary64).  xmin/xmax
// (nullable, device): the column bounds of the data S was min-max scaled
// from, which fix the corner points without a pass over S.
subkm_status subcluster_unequal_impl(subkm_ctx *ctx, const float *S, int64_t n, int32_t d,
                                     int64_t m, float *P, int32_t *perm, int64_t *offsets,
                                     double *landmarks, int32_t metric,
                                     const float *xmin = nullptr, const float *xmax = nullptr);
// Moves and objective of the local runs of the non-empty groups (run r is
// group gid[r], device array) spread over all T groups, 0 for empty ones.
subkm_status unequal_expand_local(subkm_ctx *ctx, const int32_t *gid, int R,
                                  const int32_t *it_c, const double *sse_c, int64_t T,
                                  int32_t *it, double *sse);
// Column minima and maxima of an n x d array (either output may be null);
// flag (device int) is set when a value is NaN or infinite.
subkm_status minmax_impl(subkm_ctx *ctx, const float *X, int64_t n, int32_t d, float *mins,
                         float *maxs, int *flag);
// Rounds [t0, t1) of the subclustering (segment `seg` of the caller's split;
// the segments must be launched in order on ctx->stream).
subkm_status subcluster_segment(subkm_ctx *ctx, const float *S, int64_t n, int32_t d, int64_t N,
                                int32_t landmark_mode, int32_t metric, float *P, int32_t *perm,
                                int64_t *offsets, float *landmarks, int64_t t0, int64_t t1,
                                int32_t seg);

// Lloyd runs.  `runs` is a host array; `init_mode` 0 = centers already in C,
// 1 = copy the first k points of every run into C first, 2 = strided start
// C[q] = X[q * floor(n / k)] (single-run final stage).
subkm_status lloyd_impl(subkm_ctx *ctx, const float *P, const subkm_run *runs, int32_t R,
                        float *C, int32_t *labels, int32_t max_iter, double tol,
                        int32_t precision, int32_t form, int32_t *iters, double *sse,
                        int init_mode, unsigned long long *rechecks_acc = nullptr);

// Scratch bytes per slot that a call of these sizes requests (maximum into
// req[SC_COUNT]); used for admission control.
void lloyd_scratch_requests(const subkm_run *runs, int32_t R, int32_t precision, int32_t form,
                            int32_t max_iter, int cu_count, size_t *req);
void subcluster_scratch_requests(int64_t n, int32_t d, int64_t N, size_t *req);
void unequal_scratch_requests(int64_t n, int32_t d, int64_t m, size_t *req);
size_t minmax_scratch_bytes(int64_t n, int32_t d);
// Look up this device's address of the static scratch of the
// allocation-free scaling (ctx->device current); sets ctx->noalloc_scratch.
void noalloc_scratch_init(subkm_ctx *ctx);
// Scaling with the static scratch: no allocation of any kind.
subkm_status scale_noalloc_impl(subkm_ctx *ctx, const float *X, int64_t n, int32_t d, float *S,
                                float *mins, float *maxs);
bool cluster_requests(int64_t n, int32_t d, int64_t N, int32_t k_local, int32_t k_final,
                      size_t *req);
// bytes ctx_scratch reserves for a request of `bytes`
inline size_t scratch_reserve(size_t bytes) { return bytes ? bytes + bytes / 8 + 4096 : 0; }

// ---------------------------------------------------------------------------
// Small device helpers shared by the kernels.
__device__ __forceinline__ uint32_t ordered_bits(float f) {
    // monotone map of float to uint32 (total order of non-NaN floats)
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ordered_float(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
