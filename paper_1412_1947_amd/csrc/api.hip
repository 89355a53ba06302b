// C ABI of libsubkm: argument validation, context and scratch memory, and
// the two-level method built from the stage implementations.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>

static std::mutex g_create_mu;
static std::string g_create_err;

subkm_status set_err(subkm_ctx *ctx, subkm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else {
        std::lock_guard<std::mutex> g(g_create_mu);
        g_create_err = buf;
    }
    return st;
}

void *ctx_scratch(subkm_ctx *ctx, int slot, size_t bytes) {
    ScratchBuf &b = ctx->scratch[slot];
    if (bytes == 0) bytes = 1;
    if (b.bytes >= bytes) return b.ptr;
    if (b.ptr) {
        // earlier work on the stream may still use the old buffer
        hipStreamSynchronize(ctx->stream);
        hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    const size_t want = scratch_reserve(bytes);
    if (hipMalloc(&b.ptr, want) != hipSuccess) {
        hipGetLastError();
        b.ptr = nullptr;
        set_err(ctx, SUBKM_ENOMEM, "device allocation of %zu bytes failed", want);
        return nullptr;
    }
    b.bytes = want;
    ctx->scratch_epoch += 1;
    return b.ptr;
}

void *ctx_pinned(subkm_ctx *ctx, size_t bytes) {
    if (ctx->pinned_bytes >= bytes) return ctx->pinned;
    if (ctx->pinned) {
        hipStreamSynchronize(ctx->stream);
        hipHostFree(ctx->pinned);
        ctx->pinned = nullptr;
        ctx->pinned_bytes = 0;
    }
    size_t want = std::max<size_t>(bytes, 1 << 16);
    if (hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault) != hipSuccess) {
        hipGetLastError();
        ctx->pinned = nullptr;
        set_err(ctx, SUBKM_ENOMEM, "pinned host allocation of %zu bytes failed", want);
        return nullptr;
    }
    ctx->pinned_bytes = want;
    return ctx->pinned;
}

void *ctx_stage(subkm_ctx *ctx, size_t bytes, int *slot) {
    const int q = ctx->stage_next;
    subkm_ctx::Stage &g = ctx->stage[q];
    if (!g.ev && hipEventCreateWithFlags(&g.ev, hipEventDisableTiming) != hipSuccess) {
        hipGetLastError();
        g.ev = nullptr;
        set_err(ctx, SUBKM_EDEVICE, "hipEventCreate failed");
        return nullptr;
    }
    if (g.pending) {
        // the copy issued from this slot kStageSlots calls ago
        if (hipEventSynchronize(g.ev) != hipSuccess) {
            hipGetLastError();
            set_err(ctx, SUBKM_EDEVICE, "waiting for a plan copy failed");
            return nullptr;
        }
        g.pending = false;
    }
    if (g.bytes < bytes) {
        if (g.h) hipHostFree(g.h);
        g.h = nullptr;
        g.bytes = 0;
        const size_t want = std::max<size_t>(bytes, 1 << 16);
        if (hipHostMalloc(&g.h, want, hipHostMallocDefault) != hipSuccess) {
            hipGetLastError();
            g.h = nullptr;
            set_err(ctx, SUBKM_ENOMEM, "pinned host allocation of %zu bytes failed", want);
            return nullptr;
        }
        g.bytes = want;
    }
    *slot = q;
    ctx->stage_next = (q + 1) % subkm_ctx::kStageSlots;
    return g.h;
}

subkm_status ctx_stage_issued(subkm_ctx *ctx, int slot) {
    subkm_ctx::Stage &g = ctx->stage[slot];
    SUBKM_HIP(ctx, hipEventRecord(g.ev, ctx->stream));
    g.pending = true;
    return SUBKM_OK;
}

static hipEvent_t prof_event(subkm_ctx *ctx) {
    if (!ctx->prof_free.empty()) {
        hipEvent_t e = ctx->prof_free.back();
        ctx->prof_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        hipGetLastError();
        return nullptr;
    }
    return e;
}

ProfScope::ProfScope(subkm_ctx *c, int k) : ctx(c), cls(k) {
    if (!ctx->prof_on) return;
    a = prof_event(ctx);
    if (a) hipEventRecord(a, ctx->stream);
}

ProfScope::~ProfScope() {
    if (!a) return;
    hipEvent_t b = prof_event(ctx);
    if (!b) return;
    hipEventRecord(b, ctx->stream);
    ctx->prof_pending.push_back(ProfRec{cls, a, b});
}

static void prof_resolve(subkm_ctx *ctx) {
    for (auto &r : ctx->prof_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            ctx->prof_ms[r.cls] += ms;
            ctx->prof_n[r.cls] += 1;
        }
        ctx->prof_free.push_back(r.a);
        ctx->prof_free.push_back(r.b);
    }
    ctx->prof_pending.clear();
}

// Report (and clear) what a finished launch flagged in the sticky words;
// the context's stream must be idle.
static subkm_status check_sticky(subkm_ctx *ctx) {
    int h = 0;
    SUBKM_HIP(ctx, hipMemcpy(&h, ctx->sticky, sizeof h, hipMemcpyDeviceToHost));
    if (h) {
        SUBKM_HIP(ctx, hipMemset(ctx->sticky, 0, sizeof h));
        return set_err(ctx, SUBKM_EDEVICE,
                       "a persistent Lloyd launch on this context gave up waiting at a barrier; "
                       "the results of that batched call are invalid");
    }
    return SUBKM_OK;
}

// RAII: make the context's device current for the duration of a call
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

#define CHECK_CTX(ctx)                                                                    \
    do {                                                                                  \
        if (!(ctx)) return SUBKM_EINVAL;                                                  \
        (ctx)->err.clear();                                                               \
    } while (0)

#define REQUIRE(ctx, cond, ...)                                                           \
    do {                                                                                  \
        if (!(cond)) return set_err((ctx), SUBKM_EINVAL, __VA_ARGS__);                    \
    } while (0)

extern "C" {

subkm_status subkm_create(int device, void *stream, subkm_ctx **out) {
    if (!out) return set_err(nullptr, SUBKM_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        hipGetLastError();
        return set_err(nullptr, SUBKM_EDEVICE, "no HIP device available");
    }
    if (device < 0 || device >= ndev)
        return set_err(nullptr, SUBKM_EINVAL, "device %d out of range [0,%d)", device, ndev);
    subkm_ctx *c = new (std::nothrow) subkm_ctx();
    if (!c) return set_err(nullptr, SUBKM_ENOMEM, "host allocation failed");
    c->device = device;
    c->stream = (hipStream_t)stream;
    DeviceGuard g(device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->cu_count = prop.multiProcessorCount;
    for (auto &e : c->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            hipGetLastError();
            subkm_destroy(c);
            return set_err(nullptr, SUBKM_EDEVICE, "hipEventCreate failed");
        }
    }
    if (hipMalloc(&c->sticky, 256) != hipSuccess || hipMemset(c->sticky, 0, 256) != hipSuccess) {
        hipGetLastError();
        subkm_destroy(c);
        return set_err(nullptr, SUBKM_ENOMEM, "device allocation of the context's flags failed");
    }
    noalloc_scratch_init(c);
    *out = c;
    return SUBKM_OK;
}

void subkm_destroy(subkm_ctx *ctx) {
    if (!ctx) return;
    DeviceGuard g(ctx->device);
    hipStreamSynchronize(ctx->stream);
    for (auto &b : ctx->scratch)
        if (b.ptr) hipFree(b.ptr);
    if (ctx->pinned) hipHostFree(ctx->pinned);
    for (auto &g : ctx->stage) {
        if (g.h) hipHostFree(g.h);
        if (g.ev) hipEventDestroy(g.ev);
    }
    if (ctx->sticky) hipFree(ctx->sticky);
    for (auto &e : ctx->ev)
        if (e) hipEventDestroy(e);
    prof_resolve(ctx);
    for (auto &e : ctx->prof_free) hipEventDestroy(e);
    for (auto &g : ctx->subg)
        if (g.exec) hipGraphExecDestroy(g.exec);
    if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
    delete ctx;
}

const char *subkm_last_error(const subkm_ctx *ctx) {
    if (!ctx) {
        std::lock_guard<std::mutex> g(g_create_mu);
        return g_create_err.c_str();
    }
    return ctx->err.c_str();
}

subkm_status subkm_set_stream(subkm_ctx *ctx, void *stream) {
    CHECK_CTX(ctx);
    ctx->stream = (hipStream_t)stream;
    return SUBKM_OK;
}

subkm_status subkm_synchronize(subkm_ctx *ctx) {
    CHECK_CTX(ctx);
    DeviceGuard g(ctx->device);
    SUBKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return check_sticky(ctx);
}

subkm_status subkm_tune_enable(subkm_ctx *ctx, int32_t on) {
    CHECK_CTX(ctx);
    REQUIRE(ctx, on == 0 || on == 1, "on must be 0 or 1");
    ctx->tune_on = on != 0;
    return SUBKM_OK;
}

subkm_status subkm_tune_count(subkm_ctx *ctx, int32_t *entries) {
    CHECK_CTX(ctx);
    REQUIRE(ctx, entries, "NULL array argument");
    *entries = (int32_t)ctx->tune.size();
    return SUBKM_OK;
}

static const char kTuneMagic[] = "subkm-tune 3";
static const char kTuneMagic2[] = "subkm-tune 2";  // no exchange field (0 then)
static const char kTuneMagic1[] = "subkm-tune 1";  // nor a tiles-per-block field (2 then)

subkm_status subkm_tune_save(subkm_ctx *ctx, const char *path) {
    CHECK_CTX(ctx);
    REQUIRE(ctx, path, "NULL path");
    FILE *f = std::fopen(path, "w");
    if (!f) return set_err(ctx, SUBKM_EINVAL, "cannot open %s for writing", path);
    std::fprintf(f, "%s\n", kTuneMagic);
    for (const auto &e : ctx->tune) {
        for (int i = 0; i < 5; ++i) std::fprintf(f, "%llx ", (unsigned long long)e.first.v[i]);
        std::fprintf(f, "%d %d %d %d %.6f\n", e.second.sched.gcap, e.second.sched.bdiv, e.second.sched.tpb,
                     e.second.sched.xmode, e.second.ms);
    }
    const bool ok = std::fclose(f) == 0;
    return ok ? SUBKM_OK : set_err(ctx, SUBKM_EINVAL, "cannot write %s", path);
}

subkm_status subkm_tune_load(subkm_ctx *ctx, const char *path) {
    CHECK_CTX(ctx);
    REQUIRE(ctx, path, "NULL path");
    FILE *f = std::fopen(path, "r");
    if (!f) return set_err(ctx, SUBKM_EINVAL, "cannot open %s", path);
    char head[64] = {};
    const bool read = std::fgets(head, sizeof head, f) != nullptr;
    const bool v3 = read && std::strncmp(head, kTuneMagic, sizeof kTuneMagic - 1) == 0;
    const bool v2 = read && std::strncmp(head, kTuneMagic2, sizeof kTuneMagic2 - 1) == 0;
    const bool v1 = read && std::strncmp(head, kTuneMagic1, sizeof kTuneMagic1 - 1) == 0;
    if (!v1 && !v2 && !v3) {
        std::fclose(f);
        return set_err(ctx, SUBKM_EINVAL, "%s is not a schedule file", path);
    }
    // one entry per line: five hex key words, the integer fields of the
    // format (block cap, grid divisor[, tiles per block[, exchange]]) and the
    // time; every token must parse whole
    std::map<TuneKey, TuneEntry> got;
    const int nint = v3 ? 4 : v2 ? 3 : 2;
    char line[512];
    bool bad = false;
    while (!bad && std::fgets(line, sizeof line, f)) {
        char *tok[16];
        int nt = 0;
        char *save = nullptr;
        for (char *t = strtok_r(line, " \t\r\n", &save); t; t = strtok_r(nullptr, " \t\r\n", &save)) {
            if (nt == 16) {
                bad = true;
                break;
            }
            tok[nt++] = t;
        }
        if (bad || nt == 0) continue;  // blank lines are allowed
        if (nt != 5 + nint + 1) {
            bad = true;
            continue;
        }
        TuneKey k;
        char *end = nullptr;
        for (int i = 0; i < 5 && !bad; ++i) {
            k.v[i] = std::strtoull(tok[i], &end, 16);
            bad = *end != '\0';
        }
        long iv[4] = {0, 0, 2, 0};
        for (int i = 0; i < nint && !bad; ++i) {
            iv[i] = std::strtol(tok[5 + i], &end, 10);
            bad = *end != '\0';
        }
        double ms = 0.0;
        if (!bad) {
            ms = std::strtod(tok[5 + nint], &end);
            bad = *end != '\0';
        }
        const long gcap = iv[0], bdiv = iv[1], tpb = iv[2], xmode = iv[3];
        if (bad || gcap < 1 || gcap > 1024 || bdiv < 1 || bdiv > 64 || tpb < 1 || tpb > 64 || xmode < 0 ||
            xmode > 1) {
            bad = true;
            continue;
        }
        got[k] = TuneEntry{LloydSched{(int32_t)gcap, (int32_t)bdiv, (int32_t)tpb, (int32_t)xmode}, ms};
    }
    if (bad) {
        std::fclose(f);
        return set_err(ctx, SUBKM_EINVAL, "%s: malformed entry", path);
    }
    std::fclose(f);
    for (const auto &e : got) ctx->tune[e.first] = e.second;
    return SUBKM_OK;
}

subkm_status subkm_profile_enable(subkm_ctx *ctx, int32_t on) {
    CHECK_CTX(ctx);
    DeviceGuard g(ctx->device);
    prof_resolve(ctx);
    for (int q = 0; q < PK_COUNT; ++q) {
        ctx->prof_ms[q] = 0.0;
        ctx->prof_n[q] = 0;
    }
    ctx->prof_on = on != 0;
    return SUBKM_OK;
}

subkm_status subkm_profile_query(subkm_ctx *ctx, int32_t cls, int64_t *launches, double *ms) {
    CHECK_CTX(ctx);
    REQUIRE(ctx, cls >= 0 && cls < PK_COUNT, "unknown kernel class %d", cls);
    REQUIRE(ctx, launches && ms, "NULL output");
    DeviceGuard g(ctx->device);
    prof_resolve(ctx);
    *launches = ctx->prof_n[cls];
    *ms = ctx->prof_ms[cls];
    return SUBKM_OK;
}

const char *subkm_profile_name(int32_t cls) {
    static const char *names[PK_COUNT] = {"assign", "update", "keys", "cand",
                                          "scatter", "scale", "lloyd_fused", "subcluster"};
    return (cls >= 0 && cls < PK_COUNT) ? names[cls] : "";
}

subkm_status subkm_scale(subkm_ctx *ctx, const float *X, int64_t n, int32_t d, float *S,
                         float *mins, float *maxs) {
    CHECK_CTX(ctx);
    REQUIRE(ctx, n >= 1 && n < (1ll << 31), "n must be in [1, 2^31)");
    REQUIRE(ctx, d >= 1 && d <= 4096, "d must be in [1, 4096]");
    REQUIRE(ctx, X && S && mins && maxs, "NULL array argument");
    DeviceGuard g(ctx->device);
    return scale_impl(ctx, X, n, d, S, mins, maxs, true);
}

subkm_status subkm_scale_noalloc(subkm_ctx *ctx, const float *X, int64_t n, int32_t d, float *S,
                                 float *mins, float *maxs) {
    CHECK_CTX(ctx);
    REQUIRE(ctx, n >= 1 && n < (1ll << 31), "n must be in [1, 2^31)");
    REQUIRE(ctx, d >= 1 && d <= 4096, "d must be in [1, 4096]");
    REQUIRE(ctx, X && S && mins && maxs, "NULL array argument");
    DeviceGuard g(ctx->device);
    return scale_noalloc_impl(ctx, X, n, d, S, mins, maxs);
}

subkm_status subkm_scale_colmajor(subkm_ctx *ctx, const float *X, int64_t n, int32_t d,
                                  float *S, float *mins, float *maxs) {
    CHECK_CTX(ctx);
    REQUIRE(ctx, n >= 1 && n < (1ll << 31), "n must be in [1, 2^31)");
    REQUIRE(ctx, d >= 1 && d <= 4096, "d must be in [1, 4096]");
    REQUIRE(ctx, X && S && mins && maxs, "NULL array argument");
    REQUIRE(ctx, (const void *)X != (const void *)S, "S must not alias X");
    DeviceGuard g(ctx->device);
    return scale_cm_impl(ctx, X, n, d, S, mins, maxs, true);
}

subkm_status subkm_subcluster(subkm_ctx *ctx, const float *S, int64_t n, int32_t d, int64_t N,
                              int32_t landmark_mode, int32_t metric, float *P, int32_t *perm,
                              int64_t *offsets, float *landmarks) {
    CHECK_CTX(ctx);
    REQUIRE(ctx, n >= 1 && n < (1ll << 31), "n must be in [1, 2^31)");
    REQUIRE(ctx, d >= 1 && d <= 4096, "d must be in [1, 4096]");
    REQUIRE(ctx, N >= 1, "N must be >= 1");
    REQUIRE(ctx, landmark_mode == 0 || landmark_mode == 1, "landmark_mode must be 0 or 1");
    REQUIRE(ctx, metric == SUBKM_METRIC_L2 || metric == SUBKM_METRIC_L1, "unknown metric %d",
            metric);
    REQUIRE(ctx, S && P && perm && offsets, "NULL array argument");
    REQUIRE(ctx, (const void *)S != (const void *)P, "P must not alias S");
    DeviceGuard g(ctx->device);
    return subcluster_impl(ctx, S, n, d, N, landmark_mode, metric, P, perm, offsets, landmarks);
}

subkm_status subkm_subcluster_unequal(subkm_ctx *ctx, const float *S, int64_t n, int32_t d,
                                      int64_t m, int32_t metric, float *P, int32_t *perm,
                                      int64_t *offsets, double *landmarks) {
    CHECK_CTX(ctx);
    REQUIRE(ctx, n >= 1 && n < (1ll << 31), "n must be in [1, 2^31)");
    REQUIRE(ctx, d >= 1 && d <= 4096, "d must be in [1, 4096]");
    REQUIRE(ctx, m >= 1 && m <= kUqMaxGroups, "m must be in [1, %lld]", (long long)kUqMaxGroups);
    REQUIRE(ctx, metric == SUBKM_METRIC_L2 || metric == SUBKM_METRIC_L1, "unknown metric %d",
            metric);
    REQUIRE(ctx, S && P && perm && offsets, "NULL array argument");
    REQUIRE(ctx, (const void *)S != (const void *)P, "P must not alias S");
    DeviceGuard g(ctx->device);
    return subcluster_unequal_impl(ctx, S, n, d, m, P, perm, offsets, landmarks, metric);
}

subkm_status subkm_lloyd_batched(subkm_ctx *ctx, const float *P, const subkm_run *runs,
                                 int32_t R, float *C, int32_t *labels, int32_t max_iter,
                                 double tol, int32_t precision, int32_t form, int32_t *iters,
                                 double *sse) {
    CHECK_CTX(ctx);
    REQUIRE(ctx, R >= 1, "R must be >= 1");
    REQUIRE(ctx, P && runs && C && labels && iters && sse, "NULL array argument");
    REQUIRE(ctx, max_iter >= 0, "max_iter must be >= 0");
    REQUIRE(ctx, tol >= 0 && std::isfinite(tol), "tol must be finite and >= 0");
    REQUIRE(ctx, precision == SUBKM_PREC_FP32 || precision == SUBKM_PREC_BF16,
            "unknown precision %d", precision);
    REQUIRE(ctx, form == SUBKM_FORM_BATCHED || form == SUBKM_FORM_PLAIN, "unknown form %d", form);
    for (int32_t r = 0; r < R; ++r) {
        const subkm_run &u = runs[r];
        REQUIRE(ctx, u.n >= 1 && u.n < (1ll << 31), "run %d: n must be in [1, 2^31)", r);
        REQUIRE(ctx, u.d >= 1 && u.d <= 4096, "run %d: d must be in [1, 4096]", r);
        REQUIRE(ctx, u.k >= 1 && u.k <= u.n, "run %d: k must be in [1, n]", r);
        REQUIRE(ctx, u.x_off >= 0 && u.c_off >= 0 && u.lab_off >= 0, "run %d: negative offset", r);
    }
    DeviceGuard g(ctx->device);
    return lloyd_impl(ctx, P, runs, R, C, labels, max_iter, tol, precision, form, iters, sse, 0);
}

subkm_status subkm_cluster_sizes(int64_t n, int64_t N, int32_t k_local, int64_t *T, int64_t *M) {
    if (n < 1 || N < 1 || k_local < 1 || k_local > N || !T || !M) return SUBKM_EINVAL;
    int64_t t = ceil_div(n, N);
    int64_t full = n / N, rest = n - full * N;
    int64_t m = full * (int64_t)k_local + (rest ? ceil_div(rest * (int64_t)k_local, N) : 0);
    *T = t;
    *M = m;
    return SUBKM_OK;
}

}  // extern "C"

// Scratch requests, slot by slot, of a subkm_cluster call of these sizes on
// a fresh context, for either precision and form (each slot keeps the
// largest request it sees).  False for invalid sizes.
bool cluster_requests(int64_t n, int32_t d, int64_t N, int32_t k_local, int32_t k_final,
                      size_t *req) {
    int64_t T = 0, M = 0;
    if (n < 1 || n >= (1ll << 31) || d < 1 || d > 4096 || N < 1 || k_local < 1 || k_local > N ||
        k_final < 1)
        return false;
    if (subkm_cluster_sizes(n, N, k_local, &T, &M) != SUBKM_OK || k_final > M) return false;
    // the requests of subkm_cluster, slot by slot, for either precision and
    // form (each slot keeps the largest request it has seen)
    auto need = [&](int slot, size_t b) { req[slot] = std::max(req[slot], b); };
    const size_t pts = (size_t)n * d;
    need(SC_CL_S, pts * 4);
    need(SC_CL_P, pts * 4);
    need(SC_CL_PERM, (size_t)n * 4);
    need(SC_CL_OFFS, (size_t)(T + 1) * 8);
    need(SC_CL_LOCAL, (size_t)M * d * 4);
    need(SC_CL_LLAB, (size_t)n * 4);
    need(SC_CL_LIT, (size_t)T * 4);
    need(SC_CL_LSSE, (size_t)T * 8);
    need(SC_CL_MINMAX, (size_t)d * 8);
    need(SC_CL_FINAL, (size_t)M * 4 + 128);
    need(SC_MM_PART, minmax_scratch_bytes(n, d));
    need(SC_MM_FLAG, 256);
    subcluster_scratch_requests(n, d, N, req);
    std::vector<subkm_run> runs((size_t)T);
    int64_t m = 0;
    for (int64_t t = 0; t < T; ++t) {
        const int64_t nr = std::min<int64_t>(N, n - t * N);
        runs[t] = subkm_run{t * N * d, nr, m * d, t * N, d, (int32_t)ceil_div(nr * (int64_t)k_local, N)};
        m += runs[t].k;
    }
    const subkm_run fr{0, M, 0, 0, d, k_final}, lr{0, n, 0, 0, d, k_final};
    const int big = 1 << 20;  // schedule bounded by the number of tiles
    for (int prec = 0; prec <= 1; ++prec) {
        for (int form = 0; form <= 1; ++form)
            lloyd_scratch_requests(runs.data(), (int32_t)T, prec, form, 1, big, req);
        lloyd_scratch_requests(&fr, 1, prec, SUBKM_FORM_BATCHED, 1, big, req);
        lloyd_scratch_requests(&lr, 1, prec, SUBKM_FORM_BATCHED, 0, big, req);
    }
    return true;
}

extern "C" {


size_t subkm_cluster_footprint(int64_t n, int32_t d, int64_t N, int32_t k_local,
                               int32_t k_final) {
    size_t req[SC_COUNT] = {};
    if (!cluster_requests(n, d, N, k_local, k_final, req)) return 0;
    size_t b = 0;
    for (int q = 0; q < SC_COUNT; ++q) b += scratch_reserve(req[q]);
    return b;
}

size_t subkm_device_bytes(const subkm_ctx *ctx) {
    if (!ctx) return 0;
    size_t b = 0;
    for (int q = 0; q < SC_COUNT; ++q) b += ctx->scratch[q].bytes;
    return b;
}

subkm_status subkm_cluster(subkm_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t N,
                           int32_t k_local, int32_t k_final, int32_t max_iter, double tol,
                           const subkm_opts *opts, float *centers, int32_t *labels, double *sse,
                           subkm_stats *stats) {
    CHECK_CTX(ctx);
    REQUIRE(ctx, n >= 1 && n < (1ll << 31), "n must be in [1, 2^31)");
    REQUIRE(ctx, d >= 1 && d <= 4096, "d must be in [1, 4096]");
    REQUIRE(ctx, N >= 1, "N must be >= 1");
    REQUIRE(ctx, k_local >= 1 && k_local <= N, "k_local must be in [1, N]");
    REQUIRE(ctx, max_iter >= 0, "max_iter must be >= 0");
    REQUIRE(ctx, tol >= 0 && std::isfinite(tol), "tol must be finite and >= 0");
    REQUIRE(ctx, X && centers && labels && sse, "NULL array argument");
    subkm_opts o{};
    if (opts) o = *opts;
    REQUIRE(ctx, o.landmark_mode == 0 || o.landmark_mode == 1, "landmark_mode must be 0 or 1");
    REQUIRE(ctx, o.precision == SUBKM_PREC_FP32 || o.precision == SUBKM_PREC_BF16,
            "unknown precision");
    REQUIRE(ctx, o.form == SUBKM_FORM_BATCHED || o.form == SUBKM_FORM_PLAIN, "unknown form");
    REQUIRE(ctx, o.scheme == SUBKM_SCHEME_EQUAL || o.scheme == SUBKM_SCHEME_UNEQUAL,
            "unknown scheme %d", o.scheme);
    REQUIRE(ctx, o.metric == SUBKM_METRIC_L2 || o.metric == SUBKM_METRIC_L1, "unknown metric %d",
            o.metric);
    REQUIRE(ctx, o.layout == SUBKM_LAYOUT_ROW || o.layout == SUBKM_LAYOUT_COL, "unknown layout %d",
            o.layout);
    REQUIRE(ctx, o.layout == SUBKM_LAYOUT_ROW || (const void *)X != (const void *)o.S,
            "opts->S must not alias a column-major X");
    const bool uneq = o.scheme == SUBKM_SCHEME_UNEQUAL;
    int64_t T = 0, M = 0;
    subkm_cluster_sizes(n, N, k_local, &T, &M);
    if (uneq) {
        REQUIRE(ctx, o.m >= 0, "m must be >= 0");
        T = o.m ? o.m : T;
        REQUIRE(ctx, T <= kUqMaxGroups, "m must be in [1, %lld]", (long long)kUqMaxGroups);
        // capacity: sum_r ceil(n_r k_local / N) <= floor(n k_local / N) + T, and <= n
        M = std::min<int64_t>(n, n * (int64_t)k_local / N + T);
    }
    REQUIRE(ctx, k_final >= 1 && k_final <= M, "k_final must be in [1, M=%lld]", (long long)M);
    DeviceGuard g(ctx->device);
    hipStream_t s = ctx->stream;

    const size_t pts = (size_t)n * d;
    float *S = o.S ? o.S : (float *)ctx_scratch(ctx, SC_CL_S, pts * sizeof(float));
    float *P = (float *)ctx_scratch(ctx, SC_CL_P, pts * sizeof(float));
    int32_t *perm = o.perm ? o.perm : (int32_t *)ctx_scratch(ctx, SC_CL_PERM, n * sizeof(int32_t));
    int64_t *offs = (int64_t *)ctx_scratch(ctx, SC_CL_OFFS, (T + 1) * sizeof(int64_t));
    float *loc = o.local_centers ? o.local_centers
                                 : (float *)ctx_scratch(ctx, SC_CL_LOCAL, (size_t)M * d * 4);
    int32_t *llab = (int32_t *)ctx_scratch(ctx, SC_CL_LLAB, (size_t)n * sizeof(int32_t));
    int32_t *lit = o.local_iters ? o.local_iters
                                 : (int32_t *)ctx_scratch(ctx, SC_CL_LIT, T * sizeof(int32_t));
    double *lsse = o.local_sse ? o.local_sse
                               : (double *)ctx_scratch(ctx, SC_CL_LSSE, T * sizeof(double));
    float *mm = (float *)ctx_scratch(ctx, SC_CL_MINMAX, 2 * (size_t)d * sizeof(float));
    char *fin = (char *)ctx_scratch(ctx, SC_CL_FINAL, (size_t)M * 4 + 128);
    if (!S || !P || !perm || !offs || !loc || !llab || !lit || !lsse || !mm || !fin)
        return SUBKM_ENOMEM;
    int32_t *fit = (int32_t *)fin;
    double *fsse = (double *)(fin + 16);
    unsigned long long *nrecheck = (unsigned long long *)(fin + 32);
    int32_t *flab = (int32_t *)(fin + 128);
    SUBKM_HIP(ctx, hipMemsetAsync(nrecheck, 0, sizeof(unsigned long long), s));

    hipEvent_t *ev = ctx->ev;
    if (stats) SUBKM_HIP(ctx, hipEventRecord(ev[0], s));
    if (o.layout == SUBKM_LAYOUT_COL) SUBKM_TRY(scale_cm_impl(ctx, X, n, d, S, mm, mm + d, true));
    else SUBKM_TRY(scale_impl(ctx, X, n, d, S, mm, mm + d, true));
    if (stats) SUBKM_HIP(ctx, hipEventRecord(ev[1], s));

    // local runs: one per non-empty subcluster, rows offsets[t] .. of P
    std::vector<subkm_run> runs;
    int32_t *lit_r = lit;  // moves of run r
    double *lsse_r = lsse;
    int32_t *gid_d = nullptr;  // Algorithm 2: group of run r
    auto add_run = [&](int64_t off, int64_t nr, int64_t &m) {
        subkm_run u;
        u.x_off = off * d;
        u.n = nr;
        u.c_off = m * d;
        u.lab_off = off;
        u.d = d;
        u.k = (int32_t)ceil_div(nr * (int64_t)k_local, N);
        m += u.k;
        runs.push_back(u);
    };
    if (!uneq) {
        int64_t m = 0;
        for (int64_t t = 0; t < T; ++t) add_run(t * N, std::min<int64_t>(N, n - t * N), m);
        SUBKM_TRY(subcluster_impl(ctx, S, n, d, N, o.landmark_mode, o.metric, P, perm, offs,
                                  nullptr));
        if (stats) SUBKM_HIP(ctx, hipEventRecord(ev[2], s));
    } else {
        SUBKM_TRY(subcluster_unequal_impl(ctx, S, n, d, T, P, perm, offs, nullptr, o.metric, mm,
                                          mm + d));
        if (stats) SUBKM_HIP(ctx, hipEventRecord(ev[2], s));
        // the group sizes decide the runs: read them back
        std::vector<int64_t> hoff((size_t)T + 1);
        SUBKM_HIP(ctx, hipMemcpyAsync(hoff.data(), offs, (T + 1) * sizeof(int64_t),
                                      hipMemcpyDeviceToHost, s));
        SUBKM_HIP(ctx, hipStreamSynchronize(s));
        std::vector<int32_t> gid;
        int64_t m = 0;
        for (int64_t q = 0; q < T; ++q)
            if (hoff[q + 1] > hoff[q]) {
                add_run(hoff[q], hoff[q + 1] - hoff[q], m);
                gid.push_back((int32_t)q);
            }
        M = m;
        REQUIRE(ctx, k_final <= M, "k_final must be in [1, M=%lld]", (long long)M);
        const size_t R = runs.size();
        char *lb = (char *)ctx_scratch(ctx, SC_UQ_LOCAL, R * 16 + 256);
        if (!lb) return SUBKM_ENOMEM;
        lsse_r = (double *)lb;
        lit_r = (int32_t *)(lb + R * 8);
        gid_d = (int32_t *)(lb + R * 12 + 64);
        SUBKM_HIP(ctx, hipMemcpy(gid_d, gid.data(), R * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    const int32_t R = (int32_t)runs.size();
    SUBKM_TRY(lloyd_impl(ctx, P, runs.data(), R, loc, llab, max_iter, tol, o.precision, o.form,
                         lit_r, lsse_r, 1, nrecheck));
    if (uneq) SUBKM_TRY(unequal_expand_local(ctx, gid_d, R, lit_r, lsse_r, T, lit, lsse));
    if (stats) SUBKM_HIP(ctx, hipEventRecord(ev[3], s));
    // final run on the local centers, strided start
    subkm_run fr{0, M, 0, 0, d, k_final};
    SUBKM_TRY(lloyd_impl(ctx, loc, &fr, 1, centers, flab, max_iter, tol, o.precision,
                         SUBKM_FORM_BATCHED, fit, fsse, 2, nrecheck));
    if (stats) SUBKM_HIP(ctx, hipEventRecord(ev[4], s));
    // labels of all points against the final centers (an assignment only)
    subkm_run lr{0, n, 0, 0, d, k_final};
    SUBKM_TRY(lloyd_impl(ctx, S, &lr, 1, centers, labels, 0, 0.0, o.precision,
                         SUBKM_FORM_BATCHED, fit + 1, sse, 0, nrecheck));
    if (stats) {
        SUBKM_HIP(ctx, hipEventRecord(ev[5], s));
        SUBKM_HIP(ctx, hipEventSynchronize(ev[5]));
        float ms[5];
        for (int q = 0; q < 5; ++q) SUBKM_HIP(ctx, hipEventElapsedTime(&ms[q], ev[q], ev[q + 1]));
        std::vector<int32_t> hit((size_t)R + 1);
        SUBKM_HIP(ctx, hipMemcpy(hit.data(), lit_r, R * sizeof(int32_t), hipMemcpyDeviceToHost));
        SUBKM_HIP(ctx, hipMemcpy(&hit[R], fit, sizeof(int32_t), hipMemcpyDeviceToHost));
        unsigned long long nr = 0;
        SUBKM_HIP(ctx, hipMemcpy(&nr, nrecheck, sizeof nr, hipMemcpyDeviceToHost));
        SUBKM_TRY(check_sticky(ctx));
        stats->rechecked = (int64_t)nr;
        int64_t nsel = 0;
        if (!uneq) SUBKM_TRY(subcluster_selections(ctx, S, P, n, d, N, o.metric, &nsel));
        stats->sub_selections = (int32_t)nsel;
        stats->T = T;
        stats->M = M;
        stats->final_iters = hit[R];
        int64_t lpi = 0;
        for (int32_t r = 0; r < R; ++r) lpi += runs[r].n * (int64_t)hit[r];
        stats->local_point_iters = lpi;
        stats->final_point_iters = M * (int64_t)hit[R];
        stats->us_scale = ms[0] * 1e3;
        stats->us_subcluster = ms[1] * 1e3;
        stats->us_local = ms[2] * 1e3;
        stats->us_final = ms[3] * 1e3;
        stats->us_label = ms[4] * 1e3;
        stats->us_total = (ms[0] + ms[1] + ms[2] + ms[3] + ms[4]) * 1e3;
    }
    return SUBKM_OK;
}

}  // extern "C"
