// Serving engine: clustering jobs of different n, d and k arrive while others
// run; they are admitted in arrival order as soon as a slot is idle and
// their device memory fits the budget, and the admitted jobs run on separate
// HIP streams, so their work overlaps on the device (continuous batching of
// whole jobs).  Each job is the full two-level method of subkm_cluster.
//
// Memory: every slot owns a context (stream + scratch) and a buffer set for a
// job's points and outputs; both only grow.  Before a job is admitted the
// engine computes, slot by slot and buffer by buffer, how much the job would
// add to the memory the chosen slot already holds (the same requests
// subkm_cluster makes, see cluster_requests), and admits it only if the total
// over all slots stays within the budget.  When the oldest waiting job does
// not fit, idle slots give their memory back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace {

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// bytes a buffer of `have` bytes grows by for a request of `want`
size_t growth(size_t have, size_t want) {
    const size_t r = scratch_reserve(want);
    return want > have ? r - std::min(r, have) : 0;
}

struct JobRec {
    subkm_job job;
    subkm_job_result res;
    size_t req[SC_COUNT];  // scratch requests of the call
    size_t bufs[4];        // points, labels, centers, sse
    bool done = false;
};

struct Slot {
    subkm_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    DevBuf buf[4];
    int64_t job = -1;      // running job, -1 when idle
    size_t committed = 0;  // device bytes the slot holds (idle) or may hold (running)
    std::thread th;
    std::condition_variable cv;
};

}  // namespace

struct subkm_engine {
    int device = 0;
    size_t budget = 0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_done;
    std::condition_variable cv_left;  // a waiter left subkm_engine_wait
    int waiters = 0;                  // threads inside subkm_engine_wait
    std::deque<int64_t> queue;
    std::unordered_map<int64_t, JobRec> jobs;
    int64_t next_id = 1;
    bool stop = false;
    std::chrono::steady_clock::time_point t0;
    CoopGate gate;
    std::string err;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    // bytes an idle slot holds (only its own worker changes them, and only
    // while it runs a job)
    size_t held(const Slot &s) const {
        size_t b = subkm_device_bytes(s.ctx);
        for (const DevBuf &x : s.buf) b += x.bytes;
        return b;
    }
    size_t held_total() const {
        size_t b = 0;
        for (const Slot &s : slots) b += s.committed;
        return b;
    }
    size_t grow_of(const Slot &s, const JobRec &J) const {
        size_t g = 0;
        for (int q = 0; q < SC_COUNT; ++q) g += growth(s.ctx->scratch[q].bytes, J.req[q]);
        for (int q = 0; q < 4; ++q) g += growth(s.buf[q].bytes, J.bufs[q]);
        return g;
    }
    void release(Slot &s) {
        // an idle slot gives back its memory (its stream has no work left)
        hipSetDevice(device);
        hipStreamSynchronize(s.ctx->stream);
        for (int q = 0; q < SC_COUNT; ++q) {
            ScratchBuf &b = s.ctx->scratch[q];
            if (b.ptr) hipFree(b.ptr);
            b.ptr = nullptr;
            b.bytes = 0;
        }
        s.ctx->scratch_epoch += 1;
        for (DevBuf &x : s.buf) {
            if (x.ptr) hipFree(x.ptr);
            x.ptr = nullptr;
            x.bytes = 0;
        }
        s.committed = 0;
    }
    // Admit waiting jobs in arrival order (called with mu held).
    void admit_locked() {
        while (!queue.empty()) {
            JobRec &J = jobs[queue.front()];
            int best = -1;
            size_t bg = 0;
            for (int i = 0; i < (int)slots.size(); ++i)
                if (slots[i].job < 0) {
                    const size_t g = grow_of(slots[i], J);
                    if (best < 0 || g < bg) {
                        best = i;
                        bg = g;
                    }
                }
            if (best < 0) return;  // every slot busy
            if (held_total() + bg > budget) {
                // give back the memory of the other idle slots, then retry once
                bool freed = false;
                for (int i = 0; i < (int)slots.size(); ++i)
                    if (slots[i].job < 0 && slots[i].committed > 0 && i != best) {
                        release(slots[i]);
                        freed = true;
                    }
                if (held_total() + grow_of(slots[best], J) > budget && slots[best].committed > 0) {
                    release(slots[best]);
                    freed = true;
                }
                if (!freed || held_total() + grow_of(slots[best], J) > budget) return;  // wait
            }
            const int64_t id = queue.front();
            queue.pop_front();
            J.res.t_admit = now();
            J.res.slot = best;
            slots[best].committed += grow_of(slots[best], J);
            J.res.slot_bytes_admitted = slots[best].committed;
            slots[best].job = id;
            slots[best].cv.notify_one();
        }
    }
    subkm_status run(Slot &s, JobRec &J);
    void worker(int i);
};

subkm_status subkm_engine::run(Slot &s, JobRec &J) {
    subkm_ctx *ctx = s.ctx;
    const subkm_job &j = J.job;
    for (int q = 0; q < 4; ++q) {
        DevBuf &b = s.buf[q];
        if (b.bytes < J.bufs[q]) {
            if (b.ptr) {
                hipStreamSynchronize(ctx->stream);
                hipFree(b.ptr);
            }
            b.ptr = nullptr;
            b.bytes = 0;
            const size_t want = scratch_reserve(J.bufs[q]);
            if (hipMalloc(&b.ptr, want) != hipSuccess) {
                hipGetLastError();
                b.ptr = nullptr;
                return set_err(ctx, SUBKM_ENOMEM, "device allocation of %zu bytes failed", want);
            }
            b.bytes = want;
        }
    }
    float *X = (float *)s.buf[0].ptr;
    int32_t *lab = (int32_t *)s.buf[1].ptr;
    float *cen = (float *)s.buf[2].ptr;
    double *sse = (double *)s.buf[3].ptr;
    const size_t xb = (size_t)j.n * j.d * sizeof(float);
    SUBKM_HIP(ctx, hipMemcpyAsync(X, j.X, xb, hipMemcpyHostToDevice, ctx->stream));
    subkm_opts o{};
    o.precision = j.precision;
    subkm_stats st{};
    SUBKM_TRY(subkm_cluster(ctx, X, j.n, j.d, j.N, j.k_local, j.k_final, j.max_iter, j.tol, &o, cen,
                            lab, sse, nullptr));
    SUBKM_HIP(ctx, hipMemcpyAsync(j.centers, cen, (size_t)j.k_final * j.d * sizeof(float),
                                  hipMemcpyDeviceToHost, ctx->stream));
    if (j.labels)
        SUBKM_HIP(ctx, hipMemcpyAsync(j.labels, lab, (size_t)j.n * sizeof(int32_t), hipMemcpyDeviceToHost,
                                      ctx->stream));
    double h_sse = 0.0;
    SUBKM_HIP(ctx, hipMemcpyAsync(&h_sse, sse, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    SUBKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    J.res.sse = h_sse;
    (void)st;
    return SUBKM_OK;
}

void subkm_engine::worker(int i) {
    hipSetDevice(device);
    Slot &s = slots[i];
    for (;;) {
        std::unique_lock<std::mutex> lk(mu);
        s.cv.wait(lk, [&] { return s.job >= 0 || stop; });
        if (s.job < 0) return;  // stopping
        const int64_t id = s.job;
        JobRec &J = jobs[id];
        J.res.t_start = now();
        lk.unlock();
        const subkm_status st = run(s, J);
        lk.lock();
        J.res.status = st;
        if (st != SUBKM_OK) {
            std::strncpy(J.res.message, subkm_last_error(s.ctx), sizeof J.res.message - 1);
            J.res.message[sizeof J.res.message - 1] = 0;
        }
        J.res.t_done = now();
        J.done = true;
        s.job = -1;
        s.committed = held(s);
        J.res.slot_bytes_after = s.committed;
        J.res.device_bytes = held_total();
        cv_done.notify_all();
        admit_locked();
    }
}

extern "C" {

subkm_status subkm_engine_create(int device, size_t budget_bytes, int32_t slots, subkm_engine **out) {
    if (!out || slots < 1 || slots > 16 || budget_bytes == 0) return SUBKM_EINVAL;
    *out = nullptr;
    subkm_engine *e = new subkm_engine();
    e->device = device;
    e->budget = budget_bytes;
    e->t0 = std::chrono::steady_clock::now();
    if (hipSetDevice(device) != hipSuccess ||
        hipEventCreateWithFlags(&e->gate.ev, hipEventDisableTiming) != hipSuccess) {
        hipGetLastError();
        delete e;
        return SUBKM_EDEVICE;
    }
    e->slots = std::vector<Slot>(slots);
    for (int i = 0; i < slots; ++i) {
        subkm_ctx *c = nullptr;
        hipStream_t str = nullptr;
        // one stream per slot, default priority: the slots' work overlaps
        subkm_status st = hipStreamCreateWithFlags(&str, hipStreamNonBlocking) == hipSuccess
                              ? subkm_create(device, str, &c)
                              : SUBKM_EDEVICE;
        if (st == SUBKM_OK) e->slots[i].stream = str;
        else if (str) hipStreamDestroy(str);
        if (st != SUBKM_OK) {
            for (int q = 0; q < i; ++q) {
                subkm_destroy(e->slots[q].ctx);
                hipStreamDestroy(e->slots[q].stream);
            }
            hipEventDestroy(e->gate.ev);
            delete e;
            return st;
        }
        c->coop = &e->gate;
        e->slots[i].ctx = c;
    }
    for (int i = 0; i < slots; ++i) e->slots[i].th = std::thread(&subkm_engine::worker, e, i);
    *out = e;
    return SUBKM_OK;
}

void subkm_engine_destroy(subkm_engine *e) {
    if (!e) return;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        e->stop = true;
        // jobs that were never admitted are cancelled
        for (int64_t id : e->queue) {
            JobRec &J = e->jobs[id];
            J.res.status = SUBKM_EBUSY;
            J.done = true;
        }
        e->queue.clear();
        for (Slot &s : e->slots) s.cv.notify_all();
        e->cv_done.notify_all();
    }
    for (Slot &s : e->slots)
        if (s.th.joinable()) s.th.join();
    {
        // every job is done now; threads still waiting on one leave before
        // the engine goes away
        std::unique_lock<std::mutex> lk(e->mu);
        e->cv_done.notify_all();
        e->cv_left.wait(lk, [&] { return e->waiters == 0; });
    }
    for (Slot &s : e->slots) {
        for (DevBuf &x : s.buf)
            if (x.ptr) hipFree(x.ptr);
        subkm_destroy(s.ctx);
        hipStreamDestroy(s.stream);
    }
    hipEventDestroy(e->gate.ev);
    delete e;
}

const char *subkm_engine_last_error(const subkm_engine *e) { return e ? e->err.c_str() : "null engine"; }

size_t subkm_job_footprint(const subkm_job *j) {
    if (!j) return 0;
    size_t req[SC_COUNT] = {};
    if (!cluster_requests(j->n, j->d, j->N, j->k_local, j->k_final, req)) return 0;
    size_t b = 0;
    for (int q = 0; q < SC_COUNT; ++q) b += scratch_reserve(req[q]);
    b += scratch_reserve((size_t)j->n * j->d * 4) + scratch_reserve((size_t)j->n * 4) +
         scratch_reserve((size_t)j->k_final * j->d * 4) + scratch_reserve(8);
    return b;
}

subkm_status subkm_engine_submit(subkm_engine *e, const subkm_job *job, int64_t *id) {
    if (!e || !job || !id) return SUBKM_EINVAL;
    std::lock_guard<std::mutex> lk(e->mu);
    e->err.clear();
    if (e->stop) {
        e->err = "engine is stopping";
        return SUBKM_EBUSY;
    }
    if (!job->X || !job->centers || job->max_iter < 0 || !(job->tol >= 0) ||
        (job->precision != SUBKM_PREC_FP32 && job->precision != SUBKM_PREC_BF16)) {
        e->err = "invalid job";
        return SUBKM_EINVAL;
    }
    JobRec J;
    J.job = *job;
    std::memset(&J.res, 0, sizeof J.res);
    std::memset(J.req, 0, sizeof J.req);
    if (!cluster_requests(job->n, job->d, job->N, job->k_local, job->k_final, J.req)) {
        e->err = "invalid job sizes";
        return SUBKM_EINVAL;
    }
    J.bufs[0] = (size_t)job->n * job->d * 4;
    J.bufs[1] = (size_t)job->n * 4;
    J.bufs[2] = (size_t)job->k_final * job->d * 4;
    J.bufs[3] = 8;
    const size_t fp = subkm_job_footprint(job);
    if (fp > e->budget) {
        e->err = "job needs more device memory than the engine's budget";
        return SUBKM_ENOMEM;
    }
    J.res.footprint = fp;
    J.res.slot = -1;
    J.res.t_submit = e->now();
    const int64_t k = e->next_id++;
    e->jobs.emplace(k, J);
    e->queue.push_back(k);
    *id = k;
    e->admit_locked();
    return SUBKM_OK;
}

subkm_status subkm_engine_poll(subkm_engine *e, int64_t id, int32_t *done, subkm_job_result *res) {
    if (!e || !done) return SUBKM_EINVAL;
    std::lock_guard<std::mutex> lk(e->mu);
    auto it = e->jobs.find(id);
    if (it == e->jobs.end()) return SUBKM_EINVAL;
    *done = it->second.done ? 1 : 0;
    if (it->second.done) {
        if (res) *res = it->second.res;
        e->jobs.erase(it);
    }
    return SUBKM_OK;
}

subkm_status subkm_engine_wait(subkm_engine *e, int64_t id, subkm_job_result *res) {
    if (!e) return SUBKM_EINVAL;
    std::unique_lock<std::mutex> lk(e->mu);
    auto it = e->jobs.find(id);
    if (it == e->jobs.end()) return SUBKM_EINVAL;
    e->waiters += 1;
    // the record may be taken by another thread's poll or wait meanwhile
    e->cv_done.wait(lk, [&] {
        auto f = e->jobs.find(id);
        return f == e->jobs.end() || f->second.done;
    });
    e->waiters -= 1;
    if (e->waiters == 0) e->cv_left.notify_all();
    it = e->jobs.find(id);
    if (it == e->jobs.end()) return SUBKM_EINVAL;
    if (res) *res = it->second.res;
    e->jobs.erase(it);
    return SUBKM_OK;
}

subkm_status subkm_engine_stats(subkm_engine *e, int32_t *queued, int32_t *running,
                                size_t *device_bytes) {
    if (!e) return SUBKM_EINVAL;
    std::lock_guard<std::mutex> lk(e->mu);
    if (queued) *queued = (int32_t)e->queue.size();
    int r = 0;
    for (const Slot &s : e->slots) r += s.job >= 0 ? 1 : 0;
    if (running) *running = r;
    if (device_bytes) *device_bytes = e->held_total();
    return SUBKM_OK;
}

}  // extern "C"
