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
    ap.add_argument("--cpu-runs", type=int, default=24, help="oracle Lloyd runs in the CPU sample")
    return ap.parse_args()


def assign_flops(n, d, k, assigns):
    """Algorithmic flops of `assigns` assignment passes: 2*d per point-center pair."""
    return 2.0 * d * k * n * assigns


def cpu_baseline(job, runs: int):
    """The oracle (single-threaded FP64 C) on `runs` local Lloyd runs of the
    workload's shape: n_r = N scaled points, k_local centers from the first
    k points, the same iteration limit and tolerance.  Returns the Lloyd
    point-iterations per second it achieved."""
    import oracle
    S, _, _ = oracle.scale(job.X[: runs * job.N])
    t_total, pi = 0.0, 0
    for r in range(runs):
        X = S[r * job.N:(r + 1) * job.N].astype(np.float64)
        t0 = time.perf_counter()
        out = oracle.lloyd(X, X[: job.k_local], job.max_iter, job.tol)
        t_total += time.perf_counter() - t0
        pi += job.N * out["iters"]
    return pi / t_total, t_total, pi


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build runs the method on a single MI355X "
              "(multi-GPU sharding is described in DESIGN.md, not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1412_1947_amd as subkm
    import synth

    job = synth.mid()
    n, d = job.X.shape
    X = torch.from_numpy(job.X).to("cuda:0")
    km = subkm.context(0)
    kw = dict(N=job.N, k_local=job.k_local, k_final=job.k_final, max_iter=job.max_iter, tol=job.tol)

    for _ in range(a.warmup):
        km.cluster(X, **kw)
    torch.cuda.synchronize()

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
        roofs["lloyd_fused"] = {"kernel": "k_lloyd_persist", "bound": "mfma", "achieved": ach / 1e12,
                                "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s", "frac": ach / PEAK_FP32,
                                "traffic": None, "launches": launches, "avg_launch_us": ms * 1e3 / launches,
                                "algorithmic_flops_per_step": flops_step}
    if prof.get("subcluster", (0, 0))[0]:
        launches, ms = prof["subcluster"]
        ach = sub_bytes * a.steps / (ms * 1e-3)
        roofs["subcluster"] = {"kernel": "subclustering graph", "bound": "hbm", "achieved": ach / 1e9,
                               "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": ach / PEAK_HBM,
                               "traffic": None, "launches": launches, "avg_launch_us": ms * 1e3 / launches,
                               "algorithmic_bytes_per_step": sub_bytes}
    dom = max(roofs, key=lambda c: prof[c][1]) if roofs else None
    roof = roofs.get(dom)

    # ---- plain form at matched SSE ----
    plain = None
    if not a.no_plain:
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        outp = km.cluster(X, form=subkm.FORM_PLAIN, **kw)
        torch.cuda.synchronize()
        pw = time.perf_counter() - p0
        sse_plain = float(outp["sse"].cpu()[0])
        plain = {"value": point_iters / pw, "ms_per_step": pw * 1e3, "speedup_batched": pw / (wall / a.steps),
                 "sse": sse_plain, "sse_batched": sse_batched,
                 "sse_rel_diff": abs(sse_plain - sse_batched) / sse_batched,
                 "matched": abs(sse_plain - sse_batched) <= 1e-4 * sse_batched}

    cpu = None
    if not a.no_cpu:
        rate, secs, pi = cpu_baseline(job, a.cpu_runs)
        cpu = {"value": rate, "unit": "point-iters/s", "cores": 1, "kind": "oracle",
               "sample": f"{a.cpu_runs} local Lloyd runs of the workload's shape (n_r={job.N} scaled points, "
                         f"d={d}, k={job.k_local}, <= {job.max_iter} moves, tol {job.tol}); "
                         f"{pi} point-iters in {secs:.1f} s"}

    line = {
        "metric": METRIC, "value": value, "unit": "point-iters/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "mid: n=2^20 d=16, 64 anisotropic blobs + 1% outliers; N=8192 (T=128), "
                               "k_local=256, k_final=64, <=30 moves or shift<1e-6; all local runs batched",
                   "n": n, "d": d, "N": job.N, "k_local": job.k_local, "k_final": job.k_final,
                   "max_iter": job.max_iter, "tol": job.tol, "T": T, "M": M},
        "point_iters_per_step": point_iters,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "phases_us": {k: st[k] for k in ("us_scale", "us_subcluster", "us_local", "us_final", "us_label")},
        "rechecked_assignments_per_step": st["rechecked"],
        "kernels_ms_per_step": {c: v[1] / a.steps for c, v in prof.items() if v[0]},
        "roofline": roof, "roofline_other": {c: v for c, v in roofs.items() if c != dom},
        "plain": plain, "cpu_baseline": cpu,
        "sse": sse_batched,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
