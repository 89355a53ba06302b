"""Comparison protocol of whole Lloyd runs, GPU against the oracle.

A Lloyd run is a sequence of exact decisions (every label) on inexact data
(the GPU keeps float32 centers, the oracle binary64 ones), so two correct
implementations follow the same trajectory only while no point sits on a
near tie.  The protocol therefore has two parts:

* independent trajectory: the oracle runs the run on its own, step by step,
  recording the smallest relative top-2 margin (D2 - D1) / D2 of every
  assignment and the largest center move of every update.  When that margin
  never falls to 1e-6 or below, the GPU's centers, objective and move count
  must equal the oracle's (centers and objective within 1e-5 relative; the
  move count may differ only when the oracle's move at the deciding update
  lies in [tol / 2, 2 tol], and then the two runs stopped one move of about
  tol apart, far inside the 1e-5 tolerance of the centers);
* shadow step, for every run whatever its margins: from the GPU's returned
  centers, one GPU assignment must give exactly the oracle's labels and an
  objective within 1e-5, and one GPU move must give the oracle's updated
  centers within 1e-5.

The oracle steps are C calls (ctypes releases the interpreter lock), so the
runs of a workload are spread over threads.
"""
from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np
import torch

TOL = 1e-5
NEAR_TIE = 1e-6


def threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def rel_err(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))) if a.size else 0.0


def trajectory(oracle, X64, C0, max_iter: int, tol: float) -> dict:
    """The oracle's Lloyd run (the same assign / update steps as
    oracle.lloyd) with the smallest margin of every assignment and the move
    of every update recorded."""
    C = np.array(C0, dtype=np.float64, copy=True)
    it, converged = 0, False
    shifts, margins = [], []
    while True:
        lab, sse, _, margin = oracle.assign(X64, C)
        fin = margin[np.isfinite(margin)]
        margins.append(float(fin.min()) if fin.size else np.inf)
        if it == max_iter or converged:
            break
        C, shift, _ = oracle.update(X64, lab, C)
        shifts.append(float(shift))
        it += 1
        converged = shift < tol
    return dict(centers=C, labels=lab, sse=float(sse), iters=it, shifts=shifts,
                min_margin=min(margins))


def trajectories(oracle, runs, max_iter: int, tol: float) -> list:
    """trajectory() of every (X64, C0) in `runs`, on a thread pool."""
    with cf.ThreadPoolExecutor(threads()) as ex:
        return list(ex.map(lambda r: trajectory(oracle, r[0], r[1], max_iter, tol), runs))


def iters_agree(gpu_iters: int, traj: dict, tol: float) -> bool:
    """Move counts agree, or differ only where the oracle's deciding move is
    within a factor 2 of the tolerance."""
    o = traj["iters"]
    if gpu_iters == o:
        return True
    q = min(gpu_iters, o)
    if q < 1 or q > len(traj["shifts"]):
        return False
    s = traj["shifts"][q - 1]
    return tol / 2 <= s <= 2 * tol


def check_independent(C, sse, iters, traj: dict, tol: float, what: str) -> bool:
    """Independent-trajectory part of the protocol for one run (sse None:
    the run's objective is not an output, centers and moves only).  Returns
    True when the run was compared (no near tie on the oracle's path),
    False when it is left to the shadow step."""
    if traj["min_margin"] <= NEAR_TIE:
        return False
    assert iters_agree(int(iters), traj, tol), (what, int(iters), traj["iters"], traj["shifts"][-3:])
    assert rel_err(C, traj["centers"]) <= TOL, (what, rel_err(C, traj["centers"]))
    if sse is not None:
        assert abs(float(sse) - traj["sse"]) <= TOL * traj["sse"] + 1e-300, (what, float(sse), traj["sse"])
    return True


def _gpu_batch(km, Xs, Cs, max_iter: int, precision: int):
    """One batched GPU call over runs (X float32 n x d, C float32 k x d);
    returns per-run (centers, labels), iters and objectives."""
    specs, x_off, c_off, l_off = [], 0, 0, 0
    for X, C in zip(Xs, Cs):
        n, d = X.shape
        k = C.shape[0]
        specs.append((x_off, n, c_off, l_off, d, k))
        x_off += n * d
        c_off += k * d
        l_off += n
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32).reshape(-1)).to("cuda:0")
    P = torch.cat([dev(X) for X in Xs])
    Cd = torch.cat([dev(C) for C in Cs])
    lab = torch.empty(l_off, dtype=torch.int32, device="cuda:0")
    it, sse = km.lloyd_batched(P, specs, Cd, lab, max_iter, 0.0, precision)
    torch.cuda.synchronize()
    Ch, lh, ih, sh = Cd.cpu().numpy(), lab.cpu().numpy(), it.cpu().numpy(), sse.cpu().numpy()
    out = [(Ch[co:co + k * d].reshape(k, d), lh[lo:lo + n]) for (xo, n, co, lo, d, k) in specs]
    return out, ih, sh


def shadow(km, oracle, Xs, Cs, precision: int = 0, what: str = ""):
    """Shadow step of every run (X float32, C float32 centers the GPU
    returned): one assignment with identical labels and the objective within
    1e-5; one move to the oracle's updated centers within 1e-5; labels of the
    moved centers identical again."""
    a, _, sse0 = _gpu_batch(km, Xs, Cs, 0, precision)
    b, it1, sse1 = _gpu_batch(km, Xs, Cs, 1, precision)

    def ref(j):
        X64 = Xs[j].astype(np.float64)
        C = Cs[j].astype(np.float64)
        lab0, s0, _, _ = oracle.assign(X64, C)
        Cn, _, _ = oracle.update(X64, lab0, C)
        lab1, s1, _, _ = oracle.assign(X64, b[j][0])
        return lab0, s0, Cn, lab1, s1

    with cf.ThreadPoolExecutor(threads()) as ex:
        refs = list(ex.map(ref, range(len(Xs))))
    for j, (lab0, s0, Cn, lab1, s1) in enumerate(refs):
        tag = (what, j)
        assert np.array_equal(a[j][1], lab0), tag
        assert abs(sse0[j] - s0) <= TOL * s0 + 1e-300, tag
        assert int(it1[j]) == 1, tag
        assert rel_err(b[j][0], Cn) <= TOL, (tag, rel_err(b[j][0], Cn))
        assert np.array_equal(b[j][1], lab1), tag
        assert abs(sse1[j] - s1) <= TOL * s1 + 1e-300, tag
