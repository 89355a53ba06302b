#!/usr/bin/env python3
"""Benchmark of subclustered k-means on one MI355X.

One step = the whole method on one batch of synthetic input, device-resident
before the timed region: min-max scaling, equal sized subclustering, every
local Lloyd run, the final Lloyd run on the local centers and the labelling
of all points.  Workload ("mid"): n = 2^20 points, d = 16, 64 Gaussian blobs
with anisotropic diagonal sigma U[0.2, 1.5] and 1% uniform outliers;
subclusters of N = 8192 points (128 of them), 256 local centers each, 64
final centers, at most 30 Lloyd moves or a largest center move below 1e-6.

value = Lloyd point-iterations (local + final runs) per second of whole-step
wall time.  The same step with the plain form (one local run at a time, one
launch per phase and run) is timed beside it, and its objective must match
the batched one within 1e-4 relative.  Per-kernel device times come from
HIP events the library records on its stream around every launch while the
timed steps run.  The CPU oracle is timed on a bounded sample.

Prints ONE JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Lloyd point·iters/s batched vs plain at matched SSE; p50/p99 job latency"
PEAK_FP32 = 157.3e12    # MI355X FP32 vector / matrix, FLOP/s
PEAK_BF16 = 2.5e15      # dense BF16 MFMA
PEAK_HBM = 8.0e12       # bytes/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-runs", type=int, default=4,
                    help="oracle Lloyd runs per CPU thread in the CPU sample")
    ap.add_argument("--serve-jobs", type=int, default=400, help="measured jobs of the served stream")
    ap.add_argument("--serve-warmup", type=int, default=40, help="warm-up jobs of the served stream")
    ap.add_argument("--no-serve", action="store_true", help="skip the served stream")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision workload")
    ap.add_argument("--no-ragged", action="store_true", help="skip the ragged workload")
    ap.add_argument("--no-direct", action="store_true",
                    help="skip direct Lloyd on all points (the paper's comparison baseline)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default schedules (no tuning during the warm-up)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the paper-shaped 2-D sweep")
    ap.add_argument("--no-unequal", action="store_true",
                    help="skip the Algorithm 2 measurements")
    ap.add_argument("--no-error-report", action="store_true",
                    help="skip the oracle error reports (mid and precision workloads)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a kernel of known "
                         "traffic for calibrating HBM counters)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mid_hbm_traffic.md")


def source_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1412_1947_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE, calibrated by a copy of known size), per kernel class, or {}
    when the kernels' sources (or the build script with its compiler flags)
    changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return {}
    out = {}
    for line in open(TRAFFIC_FILE):
        if line.startswith("TRAFFIC_JSON "):
            rec = json.loads(line[len("TRAFFIC_JSON "):])
            for cls, r in rec.items():
                if r.get("source_hash") == source_hash(r["sources"]):
                    out[cls] = r["bytes_per_launch"]
    return out


def assign_flops(n, d, k, assigns):
    """Algorithmic flops of `assigns` assignment passes: 2*d per point-center pair."""
    return 2.0 * d * k * n * assigns


def host_cpu():
    """Host CPU model and the cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def cpu_baseline(job, runs_per_thread: int):
    """The oracle (single-threaded FP64 C, as it stands) on local Lloyd runs
    of the workload's shape: n_r = N scaled points, k_local centers from the
    first k points, the same iteration limit and tolerance.  Timed twice:
    one run after another on one core, and P concurrent threads (P = the
    cores this process may use, at most 16) each working through its own
    runs (the oracle's C calls release the interpreter lock; the runs are
    independent, as on the GPU).  Returns both rates in Lloyd
    point-iterations per second."""
    import concurrent.futures as cf
    import oracle
    model, avail = host_cpu()
    P = max(1, min(16, avail))
    total = P * runs_per_thread
    S, _, _ = oracle.scale(job.X[: total * job.N])
    runs = [S[r * job.N:(r + 1) * job.N].astype(np.float64) for r in range(total)]

    def one(X):
        return job.N * oracle.lloyd(X, X[: job.k_local], job.max_iter, job.tol)["iters"]

    t0 = time.perf_counter()
    pi1 = sum(one(X) for X in runs[:runs_per_thread])
    t1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(P) as ex:
        piP = sum(ex.map(one, runs))
    tP = time.perf_counter() - t0
    return {"value": piP / tP, "unit": "point-iters/s", "cores": P, "kind": "oracle",
            "single_core_value": pi1 / t1, "cpu_model": model, "cpus_available": avail,
            "sample": f"{total} local Lloyd runs of the workload's shape (n_r={job.N} scaled points, "
                      f"d={job.X.shape[1]}, k={job.k_local}, <= {job.max_iter} moves, tol {job.tol}) on "
                      f"{P} threads: {piP} point-iters in {tP:.2f} s wall; single core: "
                      f"{runs_per_thread} of them, {pi1} point-iters in {t1:.2f} s"}


def mid_error_report(ref, job):
    """Error of the benchmarked results against the binary64 oracle: 8
    sampled local runs (the oracle's own run from the same start; per run the
    largest relative center difference, the relative objective difference,
    the move counts and the smallest top-2 margin on the oracle's path), the
    final run (the oracle's final stage from the GPU's local centers) and the
    objective of all points against the final centers.  A check beside the
    benchmark, outside its timed region."""
    import concurrent.futures as cf
    import oracle
    S = ref["S"].cpu().numpy()
    perm = ref["perm"].cpu().numpy()
    loc = ref["local_centers"].cpu().numpy()
    lit = ref["local_iters"].cpu().numpy()
    lsse = ref["local_sse"].cpu().numpy()
    fin = ref["centers"].cpu().numpy()
    N, k, T = job.N, job.k_local, len(lit)
    P_ = max(1, min(16, host_cpu()[1]))

    def traj(X, C0):
        C = np.array(C0, np.float64)
        it, conv, mm = 0, False, np.inf
        while True:
            lab, sse, _, margin = oracle.assign(X, C)
            f = margin[np.isfinite(margin)]
            mm = min(mm, float(f.min()) if f.size else np.inf)
            if it == job.max_iter or conv:
                return C, float(sse), it, mm
            C, shift, _ = oracle.update(X, lab, C)
            it += 1
            conv = shift < job.tol

    def rel(a, b):
        return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b))))

    sample = [int(t) for t in np.linspace(0, T - 1, 8).round()]

    def local(t):
        X = S[perm[t * N:(t + 1) * N]].astype(np.float64)
        C, sse, it, mm = traj(X, X[:k])
        return {"run": t, "max_rel_center_diff": rel(loc[t * k:(t + 1) * k], C),
                "rel_sse_diff": abs(float(lsse[t]) - sse) / sse, "moves": int(lit[t]),
                "oracle_moves": it, "oracle_min_margin": mm}

    with cf.ThreadPoolExecutor(P_) as ex:
        locs = list(ex.map(local, sample))
        M = loc.shape[0]
        Cf, _, fit, fmm = traj(loc.astype(np.float64), loc[::M // job.k_final][:job.k_final])
        chunks = [(a, min(a + (1 << 16), S.shape[0])) for a in range(0, S.shape[0], 1 << 16)]
        parts = list(ex.map(lambda ab: oracle.assign(S[ab[0]:ab[1]].astype(np.float64), fin)[:2],
                            chunks))
    labs = np.concatenate([p[0] for p in parts])
    obj = float(sum(p[1] for p in parts))
    return {"what": "binary64 oracle; local runs: the oracle's own runs from the same start; final run: "
                    "the oracle's final stage from the GPU's local centers; objective: oracle labels of all "
                    "points against the GPU's final centers",
            "local_sample": locs,
            "local_max_rel_center_diff": max(r["max_rel_center_diff"] for r in locs),
            "local_max_rel_sse_diff": max(r["rel_sse_diff"] for r in locs),
            "final_max_rel_center_diff": rel(fin, Cf), "final_moves_oracle": fit,
            "final_oracle_min_margin": fmm,
            "sse_rel_diff": abs(float(ref["sse"].cpu()[0]) - obj) / obj,
            "label_mismatches": int((ref["labels"].cpu().numpy() != labs).sum())}


def bench_direct(subkm, km, ref, job, two_level_ms):
    """The paper's comparison (Sec. VI, Table II): Lloyd directly on all n
    scaled points with k_final centers (strided start, the same rule as the
    final run), against the two-level method on the same data: SSE ratio and
    speedup."""
    import torch
    S = ref["S"]
    n, d = S.shape
    k = job.k_final
    C0 = S[torch.arange(k, device=S.device) * (n // k)].contiguous()
    C = C0.clone()
    lab = torch.empty(n, dtype=torch.int32, device="cuda:0")
    spec = [(0, n, 0, 0, d, k)]
    km.lloyd_batched(S.reshape(-1), spec, C, lab, job.max_iter, job.tol)
    times = []
    for _ in range(3):
        C.copy_(C0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, sse = km.lloyd_batched(S.reshape(-1), spec, C, lab, job.max_iter, job.tol)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ms = float(np.median(times)) * 1e3
    sse_d = float(sse.cpu()[0])
    sse_t = float(ref["sse"].cpu()[0])
    iters = int(it.cpu()[0])
    return {"what": "Lloyd on all n points, k_final centers, strided start, same stopping rule",
            "ms": ms, "iters": iters, "point_iters_per_s": n * iters / (ms * 1e-3), "sse": sse_d,
            "sse_two_level": sse_t, "sse_ratio_two_level_over_direct": sse_t / sse_d,
            "speedup_two_level": ms / two_level_ms}


def bench_unequal(subkm, km, X, ref, alg1_stats, job, kw, alg1_ms):
    """Algorithm 2 (Sec. III) on the same workload: the subclustering call on
    its own against the HBM roofline (algorithmic bytes: read S, write P and
    perm), and the whole method with it next to Algorithm 1."""
    import torch
    S = ref["S"]
    n, d = S.shape
    m = -(-n // job.N)
    km.subcluster_unequal(S, m)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    torch.cuda.synchronize()
    for k in range(5):
        ev[k].record()
        km.subcluster_unequal(S, m)
    ev[5].record()
    torch.cuda.synchronize()
    sub_ms = float(np.median([ev[k].elapsed_time(ev[k + 1]) for k in range(5)]))
    nbytes = n * d * 4 * 2 + n * 4
    ach = nbytes / (sub_ms * 1e-3)
    out = km.cluster(X, scheme=subkm.SCHEME_UNEQUAL, stats=True, **kw)
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = km.cluster(X, scheme=subkm.SCHEME_UNEQUAL, stats=True, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    st = out["stats"]
    ms = float(np.median(times)) * 1e3
    sse = float(out["sse"].cpu()[0])
    _, _, offs = km.subcluster_unequal(S, m)
    sizes = np.diff(offs.cpu().numpy())
    # a group of n_g points gets ceil(n_g k_local / N) local centers, so one
    # move of the local runs costs sum_g 2 d n_g k_g flops: it grows with the
    # square of the group sizes, against 2 d n k_local for N-point groups
    kg = -(-sizes * job.k_local // job.N)
    gflop_move = float((2.0 * d * sizes * kg).sum()) / 1e9
    gflop_move_alg1 = 2.0 * d * n * job.k_local / 1e9
    return {"what": "Algorithm 2: m landmarks on the segment from the min to the max corner, "
                    "nearest-landmark groups", "m": m,
            "subcluster_ms": sub_ms, "subcluster_gbps": ach / 1e9,
            "subcluster_roofline": {"bound": "hbm", "achieved": ach / 1e9, "peak": PEAK_HBM / 1e9,
                                    "unit": "GB/s", "frac": ach / PEAK_HBM,
                                    "algorithmic_bytes": nbytes},
            "alg1_subcluster_ms": alg1_stats["us_subcluster"] * 1e-3,
            "group_sizes": {"min": int(sizes.min()), "max": int(sizes.max()),
                            "empty": int((sizes == 0).sum())},
            "local_gflop_per_move": gflop_move, "alg1_local_gflop_per_move": gflop_move_alg1,
            "ms_per_step": ms, "alg1_ms_per_step": alg1_ms, "M": st["M"],
            "point_iters_per_step": int(st["local_point_iters"] + st["final_point_iters"]),
            "phases_us": {k: st[k] for k in ("us_scale", "us_subcluster", "us_local", "us_final",
                                            "us_label")},
            "sse": sse, "alg1_sse": float(ref["sse"].cpu()[0])}


# Sec. VI Tables II and III (seconds on a Tesla C2075 with a Xeon E5-1410 host):
# traditional / parallel k-means at 100k, 250k, 500k points, and the parallel
# time at compression values 5, 10, 15 (the cell for 20 is empty)
PAPER_TABLE2 = {100_000: (2.328, 2.78), 250_000: (25.6, 4.96), 500_000: (156.8, 6.2)}
PAPER_TABLE3 = {5: 6.2, 10: 5.76, 15: 4.83, 20: None}


def bench_paper_sweep(subkm, km, synth):
    """The shape of the paper's timing experiment: 2-D blobs with 500 points
    per cluster (k_final = n / 500), Lloyd on all points against the
    two-level method (Algorithm 1, subclusters of N = 10000 points, compression
    c = N / k_local), at n = 100k, 250k, 500k with c = 5, and c = 5..20 at
    500k.  Both use <= 30 moves or a move below 1e-6."""
    import torch
    N, max_iter, tol = 10_000, 30, 1e-6

    def timed(fn, reps=2):
        fn()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)) * 1e3, out

    rows, sweep = [], []
    for n in (100_000, 250_000, 500_000):
        X = torch.from_numpy(synth.paper2d(n)).to("cuda:0")
        k = n // 500
        S = km.scale(X)[0]
        C0 = S[torch.arange(k, device=S.device) * (n // k)].contiguous()
        C = C0.clone()
        lab = torch.empty(n, dtype=torch.int32, device="cuda:0")

        def direct():
            C.copy_(C0)
            return km.lloyd_batched(S.reshape(-1), [(0, n, 0, 0, 2, k)], C, lab, max_iter, tol)

        ms_d, (it_d, sse_d) = timed(direct)
        cs = (5, 10, 15, 20) if n == 500_000 else (5,)
        for c in cs:
            def two_level():
                return km.cluster(X, N=N, k_local=N // c, k_final=k, max_iter=max_iter, tol=tol)
            ms_t, out = timed(two_level)
            sse_t = float(out["sse"].cpu()[0])
            rec = {"n": n, "k_final": k, "c": c, "N": N, "k_local": N // c, "two_level_ms": ms_t,
                   "sse": sse_t}
            if c == 5:
                rows.append(dict(rec, direct_ms=ms_d, direct_iters=int(it_d.cpu()[0]),
                                 direct_sse=float(sse_d.cpu()[0]), speedup=ms_d / ms_t,
                                 sse_ratio=sse_t / float(sse_d.cpu()[0]),
                                 paper_s={"traditional": PAPER_TABLE2[n][0],
                                          "parallel": PAPER_TABLE2[n][1]}))
            if n == 500_000:
                sweep.append(dict(rec, speedup_over_direct=ms_d / ms_t, paper_s=PAPER_TABLE3[c]))
        del X, S, C, C0, lab
    return {"what": "2-D blobs, 500 points per cluster; direct Lloyd vs the two-level method "
                    "(paper numbers: seconds on a Tesla C2075, context only)",
            "table2": rows, "table3": sweep}


def bench_serving(subkm, synth, a):
    """Poisson stream at 50 jobs/s through the serving engine (4 slots, 200 GB
    budget); latency = completion - scheduled arrival; jobs take their points
    from per-d pools in pinned host memory (the copy to the GPU is part of the
    latency)."""
    import threading
    import torch
    n_max = 2_000_000
    pools = {d: torch.from_numpy(X).pin_memory() for d, X in synth.serving_pool(n_max=n_max).items()}
    reqs = synth.serving_stream(a.serve_warmup + a.serve_jobs, rate_hz=50.0)
    eng = subkm.Engine(0, budget_bytes=200 << 30, slots=4)
    done = {}
    ids = []
    lock = threading.Lock()

    def collect():
        i = 0
        while True:
            with lock:
                if i >= len(reqs):
                    return
                have = i < len(ids)
                jid = ids[i] if have else None
            if not have:
                time.sleep(0.0005)
                continue
            done[i] = eng.wait(jid)
            i += 1

    th = threading.Thread(target=collect)
    th.start()
    t0 = time.perf_counter()
    late = []
    for r in reqs:
        wait = t0 + r.arrival_s - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        off, n = synth.pool_slice(r, n_max)
        X = pools[r.d][off:off + n]
        sub = time.perf_counter()
        jid = eng.submit(X, 8192, 256, r.k_final, 30, 1e-6)
        late.append(max(0.0, sub - (t0 + r.arrival_s)))
        with lock:
            ids.append(jid)
    th.join()
    eng.close()
    meas = range(a.serve_warmup, len(reqs))
    lat = np.array([(done[i]["t_done"] - done[i]["t_submit"] + late[i]) * 1e3 for i in meas])
    qwait = np.array([(done[i]["t_admit"] - done[i]["t_submit"]) * 1e3 for i in meas])
    first = min(done[i]["t_submit"] - late[i] for i in meas)
    last = max(done[i]["t_done"] for i in meas)
    pts = sum(reqs[i].n for i in meas)
    # concurrency: largest number of jobs running at once
    ev = sorted([(done[i]["t_start"], 1) for i in meas] + [(done[i]["t_done"], -1) for i in meas])
    cur = peak = 0
    for _, e in ev:
        cur += e
        peak = max(peak, cur)
    return {"jobs": len(lat), "warmup_jobs": a.serve_warmup, "rate_hz": 50.0,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
            "queue_wait_p99_ms": float(np.percentile(qwait, 99)),
            "points_per_s": pts / (last - first), "makespan_s": last - first,
            "peak_concurrent_jobs": peak, "slots": 4, "budget_gb": 200,
            "peak_device_gb": max(done[i]["device_bytes"] for i in meas) / 1e9,
            "workload": "Poisson 50 jobs/s; n log-uniform [1e4, 2e6]; d in {4,8,16,32,64}; k_final U[8,256]; "
                        "N=8192, k_local=256, <=30 moves or shift<1e-6; points from per-d blob pools"}


def bench_precision(subkm, synth, a):
    """Precision workload (n = 2^22, d = 128, 256 blobs, N = 32768, 1024
    local and 256 final centers): whole method with split-bfloat16 and with
    float32 matrix-core distances; both give the exact labels, so the results
    must coincide.  Roofline of the split assignment against bf16 peak."""
    import torch
    job = synth.precision()
    n, d = job.X.shape
    X = torch.from_numpy(job.X).to("cuda:0")
    km = subkm.context(0)
    kw = dict(N=job.N, k_local=job.k_local, k_final=job.k_final, max_iter=job.max_iter, tol=job.tol)
    out = {}
    for name, prec in (("bf16", subkm.PREC_BF16), ("fp32", subkm.PREC_FP32)):
        ref = km.cluster(X, precision=prec, intermediates=True, stats=True, **kw)
        # phase times from a call with the timed calls' buffers (no graph capture in it)
        st_warm = km.cluster(X, precision=prec, stats=True, **kw)["stats"]
        km.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 2
        for _ in range(reps):
            km.cluster(X, precision=prec, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        prof = km.profile_read()
        km.profile(False)
        st = ref["stats"]
        T, M = st["T"], st["M"]
        lit = ref["local_iters"].cpu().numpy()
        assigns = int(lit.sum()) + T
        flops = 2.0 * d * job.k_local * job.N * assigns          # local assignments
        flops += 2.0 * d * job.k_final * M * (st["final_iters"] + 1) + 2.0 * d * job.k_final * n
        pi = st["local_point_iters"] + st["final_point_iters"]
        a_launch, a_ms = prof.get("assign", (0, 0.0))
        out[name] = {"ms_per_step": ms, "point_iters_per_s": pi / (ms * 1e-3),
                     "sse": float(ref["sse"].cpu()[0]), "phases_us": {k: st_warm[k] for k in (
                         "us_scale", "us_subcluster", "us_local", "us_final", "us_label")},
                     "rechecked_fraction": st["rechecked"] / (n * 1.0 * (assigns / T) + M * (st["final_iters"] + 1)),
                     "assign_ms_per_step": a_ms / reps,
                     "assign_achieved_tflops": flops / (a_ms / reps * 1e-3) / 1e12}
        out[name]["_ref"] = ref
    b, f = out["bf16"], out["fp32"]
    same = (b["sse"] == f["sse"] and torch.equal(b["_ref"]["centers"], f["_ref"]["centers"])
            and torch.equal(b["_ref"]["labels"], f["_ref"]["labels"]))
    ach = b["assign_achieved_tflops"] * 1e12
    res = {"workload": "n=2^22 d=128, 256 blobs (sigma 1, means N(0,25 I)); N=32768 (T=128), k_local=1024, "
                       "k_final=256, <=30 moves or shift<1e-6",
           "bf16_ms_per_step": b["ms_per_step"], "fp32_ms_per_step": f["ms_per_step"],
           "speedup_bf16": f["ms_per_step"] / b["ms_per_step"],
           "bf16_point_iters_per_s": b["point_iters_per_s"],
           "identical_results": bool(same), "sse": b["sse"],
           "phases_us_bf16": b["phases_us"], "phases_us_fp32": f["phases_us"],
           "rechecked_fraction_bf16": b["rechecked_fraction"], "rechecked_fraction_fp32": f["rechecked_fraction"],
           "assign_roofline_bf16": {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAK_BF16 / 1e12,
                                    "unit": "TFLOP/s", "frac": ach / PEAK_BF16,
                                    "note": "algorithmic 2dk flops per point-assignment; the split form "
                                            "issues three bf16 products per algorithmic one"},
           "assign_fp32_achieved_tflops": f["assign_achieved_tflops"]}
    if not a.no_error_report:
        res["error_vs_oracle"] = precision_error_report(subkm, b["_ref"], job)
    return res


def precision_error_report(subkm, ref, job):
    """Error of the precision workload's results against the binary64
    oracle, one Lloyd move from the same float32 centers (a whole oracle run
    at k = 1024, d = 128 is about 10^11 operations per run): 4 sampled local
    runs (from the GPU's returned local centers) and the final run (from the
    GPU's final centers, on the GPU's local centers), each on the GPU
    (split-bfloat16) and in the oracle: label mismatches, largest center
    difference, relative objective difference; and the objective of all
    points against the final centers.  A check beside the benchmark."""
    import concurrent.futures as cf
    import torch
    import oracle
    S = ref["S"]
    perm = ref["perm"].cpu().numpy()
    loc = ref["local_centers"].cpu().numpy()
    fin = ref["centers"].cpu().numpy()
    N, k, d = job.N, job.k_local, int(S.shape[1])
    T = perm.shape[0] // N
    P_ = max(1, min(16, host_cpu()[1]))

    def one_move(X32, C0):
        n, kk = X32.shape[0], C0.shape[0]
        Cd = torch.from_numpy(C0.copy()).to("cuda:0")
        lab = torch.empty(n, dtype=torch.int32, device="cuda:0")
        _, sse = subkm.lloyd_batched(torch.from_numpy(X32).to("cuda:0").reshape(-1),
                                     [(0, n, 0, 0, d, kk)], Cd, lab, 1, 0.0, precision=subkm.PREC_BF16)
        Cg, lg, sg = Cd.cpu().numpy(), lab.cpu().numpy(), float(sse.cpu()[0])
        X64 = X32.astype(np.float64)
        lab0, _, _, _ = oracle.assign(X64, C0)
        C1, _, _ = oracle.update(X64, lab0, C0.astype(np.float64))
        lab1, sse1, _, margin = oracle.assign(X64, Cg)
        return {"n": n, "k": kk,
                "max_abs_center_diff": float(np.abs(Cg - C1).max()),
                "max_rel_center_diff": float(np.max(np.abs(Cg - C1) / np.maximum(1.0, np.abs(C1)))),
                "label_mismatches": int((lg != lab1).sum()),
                "rel_sse_diff": float(abs(sg - sse1) / sse1),
                "near_ties_below_1e-6": int(np.sum(np.isfinite(margin) & (margin < 1e-6)))}

    S_h = S.cpu().numpy()
    sample = [0, T // 3, 2 * T // 3, T - 1]
    locs = []
    for t in sample:
        X32 = np.ascontiguousarray(S_h[perm[t * N:(t + 1) * N]])
        locs.append(dict(one_move(X32, loc[t * k:(t + 1) * k].copy()), run=t))
    final = one_move(loc, fin.copy())
    chunks = [(a, min(a + (1 << 16), S_h.shape[0])) for a in range(0, S_h.shape[0], 1 << 16)]
    with cf.ThreadPoolExecutor(P_) as ex:
        parts = list(ex.map(lambda ab: oracle.assign(S_h[ab[0]:ab[1]].astype(np.float64), fin)[:2],
                            chunks))
    labs = np.concatenate([p[0] for p in parts])
    obj = float(sum(p[1] for p in parts))
    return {"what": "one move from the same float32 centers on the GPU (split-bfloat16) and in the binary64 "
                    "oracle; objective: oracle labels of all points against the GPU's final centers",
            "d": d, "local_sample": locs, "final": final,
            "sse_rel_diff": abs(float(ref["sse"].cpu()[0]) - obj) / obj,
            "label_mismatches": int((ref["labels"].cpu().numpy() != labs).sum())}


def bench_ragged(subkm, synth, a):
    """512 independent runs, sizes log-uniform in [1k, 64k], d in {8, 32},
    k = min(ceil(n/32), 1024), each min-max scaled on its own; all runs in
    one batched call (<= 30 moves or shift < 1e-6)."""
    import torch
    rs = synth.ragged()
    km = subkm.context(0)
    parts, specs, cinit = [], [], []
    x_off = c_off = l_off = 0
    for X, k in zip(rs.X, rs.k):
        S, _, _ = km.scale(torch.from_numpy(X).to("cuda:0"))
        n, d = S.shape
        parts.append(S.reshape(-1))
        cinit.append(S[:k].reshape(-1))
        specs.append((x_off, n, c_off, l_off, d, k))
        x_off += n * d
        c_off += k * d
        l_off += n
    P = torch.cat(parts)
    C0 = torch.cat(cinit)
    C = C0.clone()
    lab = torch.empty(l_off, dtype=torch.int32, device="cuda:0")
    it, sse = km.lloyd_batched(P, specs, C, lab, rs.max_iter, rs.tol)
    times = []
    for _ in range(3):
        C.copy_(C0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, sse = km.lloyd_batched(P, specs, C, lab, rs.max_iter, rs.tol)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ms = float(np.median(times)) * 1e3
    its = it.cpu().numpy()
    pi = sum(sp[1] * int(i) for sp, i in zip(specs, its))
    flops = sum(2.0 * sp[4] * sp[5] * sp[1] * (int(i) + 1) for sp, i in zip(specs, its))
    return {"workload": "512 runs, n log-uniform [1024, 65536], d in {8,32}, k=min(ceil(n/32),1024), "
                        "<=30 moves or shift<1e-6, one batched call",
            "runs": len(specs), "points": l_off, "ms_per_call": ms, "point_iters_per_s": pi / (ms * 1e-3),
            "achieved_tflops": flops / (ms * 1e-3) / 1e12, "frac_fp32_peak": flops / (ms * 1e-3) / PEAK_FP32,
            "iters_mean": float(its.mean())}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the method runs on a single MI355X; sharding "
              "across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1412_1947_amd as subkm
    import synth

    if a.copy_calib_mib:
        src = torch.empty(a.copy_calib_mib << 18, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    job = synth.mid()
    n, d = job.X.shape
    X = torch.from_numpy(job.X).to("cuda:0")
    km = subkm.context(0)
    kw = dict(N=job.N, k_local=job.k_local, k_final=job.k_final, max_iter=job.max_iter, tol=job.tol)

    # the schedule tuner picks the batched form's schedules during the warm-up
    # (never inside the timed region; results do not depend on it)
    tune = a.warmup > 0 and not a.no_tune
    km.tune(tune)
    for _ in range(a.warmup):
        km.cluster(X, **kw)
    torch.cuda.synchronize()
    km.tune(False)

    # work of one step (deterministic: every step does exactly the same)
    ref = km.cluster(X, intermediates=True, stats=True, **kw)
    st = ref["stats"]
    T, M = st["T"], st["M"]
    lit = ref["local_iters"].cpu().numpy()
    kr = [-(-min(job.N, n - t * job.N) * job.k_local // job.N) for t in range(T)]
    nr = [min(job.N, n - t * job.N) for t in range(T)]
    point_iters = int(st["local_point_iters"] + st["final_point_iters"])
    flops_step = sum(assign_flops(nr[t], d, kr[t], int(lit[t]) + 1) for t in range(T))
    flops_step += assign_flops(M, d, job.k_final, st["final_iters"] + 1)
    flops_step += assign_flops(n, d, job.k_final, 1)
    sse_batched = float(ref["sse"].cpu()[0])
    # phase times from a call with the timed steps' buffers (the call above
    # asks for intermediates in new buffers, which captures a new
    # subclustering graph and would count the capture in its phase)
    st_warm = km.cluster(X, stats=True, **kw)["stats"]

    # ---- timed region: K steps, per-launch kernel events on ----
    km.profile(True)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        starts[s].record()
        km.cluster(X, **kw)
        ends[s].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = km.profile_read()
    km.profile(False)
    lat = np.array([starts[s].elapsed_time(ends[s]) for s in range(a.steps)])
    ms_per_step = wall / a.steps * 1e3
    value = point_iters / (wall / a.steps)

    # rooflines: the Lloyd kernels (FP32 matrix cores) and the subclustering
    # graph (HBM); the dominant one (largest device time) is reported first
    sub_bytes = 0
    nrem = n
    for t in range(T):
        sub_bytes += nrem * d * 4          # every remaining point is read once per round
        nrem -= min(job.N, nrem)
    sub_bytes += n * d * 4                 # and every point is written once to its subcluster
    roofs = {}
    if prof.get("lloyd_fused", (0, 0))[0]:
        launches, ms = prof["lloyd_fused"]
        ach = flops_step * a.steps / (ms * 1e-3)
        # the distances are float32-class (every label is certified exact), so
        # the algorithmic flops are priced at the FP32 matrix peak; for d = 8,
        # 16, 32 the kernel executes them as split-bfloat16 products (four
        # bfloat16 products per float32 one, ceil(k/16) blocks of 16 centers),
        # whose issue rate is reported against the BF16 peak beside it
        issued = 4.0 * flops_step if d in (8, 16, 32) else None
        roofs["lloyd_fused"] = {"kernel": "k_lloyd_persist", "bound": "mfma", "achieved": ach / 1e12,
                                "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s", "frac": ach / PEAK_FP32,
                                "traffic": None, "launches": launches, "avg_launch_us": ms * 1e3 / launches,
                                "algorithmic_flops_per_step": flops_step,
                                "executed": None if issued is None else {
                                    "instruction": "v_mfma_f32_16x16x32_bf16 (split bf16, f32 accumulate)",
                                    "issued_flops_per_step": issued,
                                    "achieved": issued * a.steps / (ms * 1e-3) / 1e12,
                                    "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s",
                                    "frac": issued * a.steps / (ms * 1e-3) / PEAK_BF16}}
    if prof.get("subcluster", (0, 0))[0]:
        launches, ms = prof["subcluster"]
        ach = sub_bytes * a.steps / (ms * 1e-3)
        roofs["subcluster"] = {"kernel": "subclustering graph", "bound": "hbm", "achieved": ach / 1e9,
                               "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": ach / PEAK_HBM,
                               "traffic": None, "launches": launches, "avg_launch_us": ms * 1e3 / launches,
                               "algorithmic_bytes_per_step": sub_bytes}
    traffic = measured_traffic()
    for c, r in roofs.items():
        r["traffic"] = traffic.get(c)
    dom = max(roofs, key=lambda c: prof[c][1]) if roofs else None
    roof = roofs.get(dom)

    # ---- plain form at matched SSE: one untimed call, then the median of 3 ----
    plain = None
    if not a.no_plain:
        km.cluster(X, form=subkm.FORM_PLAIN, **kw)
        pts = []
        for _ in range(3):
            torch.cuda.synchronize()
            p0 = time.perf_counter()
            outp = km.cluster(X, form=subkm.FORM_PLAIN, **kw)
            torch.cuda.synchronize()
            pts.append(time.perf_counter() - p0)
        pw = float(np.median(pts))
        sse_plain = float(outp["sse"].cpu()[0])
        plain = {"value": point_iters / pw, "ms_per_step": pw * 1e3,
                 "ms_samples": [t * 1e3 for t in pts], "speedup_batched": pw / (wall / a.steps),
                 "sse": sse_plain, "sse_batched": sse_batched,
                 "sse_rel_diff": abs(sse_plain - sse_batched) / sse_batched,
                 "matched": abs(sse_plain - sse_batched) <= 1e-4 * sse_batched}

    cpu = None if a.no_cpu else cpu_baseline(job, a.cpu_runs)
    err = None if a.no_error_report else mid_error_report(ref, job)

    direct = None if a.no_direct else bench_direct(subkm, km, ref, job, ms_per_step)
    unequal = None if a.no_unequal else bench_unequal(subkm, km, X, ref, st_warm, job, kw, ms_per_step)
    sweep = None if a.no_sweep else bench_paper_sweep(subkm, km, synth)
    serving = None if a.no_serve else bench_serving(subkm, synth, a)
    precision = None if a.no_precision else bench_precision(subkm, synth, a)
    ragged = None if a.no_ragged else bench_ragged(subkm, synth, a)

    line = {
        "metric": METRIC, "value": value, "unit": "point-iters/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "dtype_note": ("float32 data and centers; assignment distances on split-bfloat16 matrix "
                       "cores with float32 accumulation (float32 matrix cores for uncertain points, "
                       "binary64 for the final decision), int64 center sums, binary64 keys and "
                       "objective"),
        "config": {"workload": "mid: n=2^20 d=16, 64 anisotropic blobs + 1% outliers; N=8192 (T=128), "
                               "k_local=256, k_final=64, <=30 moves or shift<1e-6; all local runs batched",
                   "n": n, "d": d, "N": job.N, "k_local": job.k_local, "k_final": job.k_final,
                   "max_iter": job.max_iter, "tol": job.tol, "T": T, "M": M},
        "point_iters_per_step": point_iters,
        "latency_ms": ({"p50": serving["p50_ms"], "p99": serving["p99_ms"], "of": "served job stream"}
                       if serving else None),
        "step_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "phases_us": {k: st_warm[k] for k in ("us_scale", "us_subcluster", "us_local", "us_final",
                                              "us_label")},
        "rechecked_assignments_per_step": st["rechecked"],
        "subcluster_selection_passes": st["sub_selections"],
        "tuned_shapes": km.tuned(),
        "kernels_ms_per_step": {c: v[1] / a.steps for c, v in prof.items() if v[0]},
        "roofline": roof, "roofline_other": {c: v for c, v in roofs.items() if c != dom},
        "plain": plain, "cpu_baseline": cpu,
        "sse": sse_batched, "error_vs_oracle": err,
        "direct": direct, "unequal": unequal, "paper_sweep": sweep, "serving": serving, "precision": precision, "ragged": ragged,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
