"""CPU oracle for subclustered k-means -- TEST INFRASTRUCTURE ONLY.

A plain, single-threaded FP64 reference written from the paper ("A parallel
sampling based clustering", arXiv 1412.1947): min-max scaling, equal sized
subclustering (Sec. II, Algorithm 1), unequal sized subclustering (Sec. III,
Algorithm 2), Lloyd's algorithm inside every
subcluster and on the local centers (Sec. I, Sec. V).  The arithmetic lives
in ``subkm_oracle.c``; this module only compiles it with gcc and marshals
numpy arrays.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import it; the HIP library never does.

Parity status of every function is pinned by ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "subkm_oracle.c")
_LIB = os.path.join(_HERE, "libsubkm_oracle.so")
_CFLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (IEEE binary64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
            lib.subkm_ref_scale.argtypes = [P, i64, i32, P, P, P]
            lib.subkm_ref_scale.restype = ctypes.c_int
            lib.subkm_ref_subcluster.argtypes = [P, i64, i32, i64, i32, i32, P, P, P]
            lib.subkm_ref_subcluster.restype = i64
            lib.subkm_ref_assign.argtypes = [P, i64, i32, i32, P, P, P, P]
            lib.subkm_ref_assign.restype = f64
            lib.subkm_ref_update.argtypes = [P, i64, i32, i32, P, P, P, P]
            lib.subkm_ref_update.restype = f64
            lib.subkm_ref_lloyd.argtypes = [P, i64, i32, i32, P, i32, f64, P, P, P, P]
            lib.subkm_ref_lloyd.restype = i32
            lib.subkm_ref_subcluster_unequal.argtypes = [P, i64, i32, i64, i32, P, P, P, P]
            lib.subkm_ref_subcluster_unequal.restype = i64
            lib.subkm_ref_cluster.argtypes = [P, i64, i32, i64, i32, i32, i32, f64, i32, i32,
                                              i64, i32, P, P, P, P, P, P, P, P, P, P, P, P, P]
            lib.subkm_ref_cluster.restype = ctypes.c_int
            _lib = lib
    return _lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(X):
    return np.ascontiguousarray(X, dtype=np.float32)


def _f64(X):
    return np.ascontiguousarray(X, dtype=np.float64)


def scale(X):
    """Min-max scaling. Returns (S, mins, maxs); raises ValueError on NaN/Inf."""
    X = _f32(X)
    n, d = X.shape
    S = np.empty_like(X)
    mins = np.empty(d, np.float32)
    maxs = np.empty(d, np.float32)
    if _load().subkm_ref_scale(_p(X), n, d, _p(S), _p(mins), _p(maxs)) != 0:
        raise ValueError("non-finite input")
    return S, mins, maxs


def subcluster(S, N: int, fixed_landmark: bool = False, metric: int = 0):
    """Algorithm 1 (metric 0: squared Euclidean, 1: Manhattan similarity).
    Returns (perm int64[n], offsets int64[T+1], landmarks f32[T,d])."""
    S = _f32(S)
    n, d = S.shape
    T_cap = -(-n // N)
    perm = np.empty(n, np.int64)
    offsets = np.empty(T_cap + 1, np.int64)
    lms = np.empty((T_cap, d), np.float32)
    T = _load().subkm_ref_subcluster(_p(S), n, d, int(N), int(fixed_landmark), int(metric),
                                     _p(perm), _p(offsets), _p(lms))
    if T < 0:
        raise ValueError("invalid arguments")
    return perm, offsets[:T + 1].copy(), lms[:T].copy()


def subcluster_unequal(S, m: int, metric: int = 0):
    """Algorithm 2 (metric as for subcluster). Returns (perm int64[n],
    offsets int64[m+1], landmarks f64[m,d], group int32[n])."""
    S = _f32(S)
    n, d = S.shape
    perm = np.empty(n, np.int64)
    offsets = np.empty(m + 1, np.int64)
    lms = np.empty((m, d), np.float64)
    grp = np.empty(n, np.int32)
    T = _load().subkm_ref_subcluster_unequal(_p(S), n, d, int(m), int(metric), _p(perm),
                                             _p(offsets), _p(lms), _p(grp))
    if T < 0:
        raise ValueError("invalid arguments")
    return perm, offsets, lms, grp


def assign(X, C):
    """Assignment step. Returns (labels, sse, dmin, margin)."""
    X = _f64(X)
    C = _f64(C)
    n, d = X.shape
    k = C.shape[0]
    lab = np.empty(n, np.int32)
    dmin = np.empty(n, np.float64)
    margin = np.empty(n, np.float64)
    sse = _load().subkm_ref_assign(_p(X), n, d, k, _p(C), _p(lab), _p(dmin), _p(margin))
    return lab, sse, dmin, margin


def update(X, labels, C):
    """Update step. Returns (C_new, shift, counts)."""
    X = _f64(X)
    C = _f64(C)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    n, d = X.shape
    k = C.shape[0]
    out = np.empty_like(C)
    cnt = np.empty(k, np.int64)
    shift = _load().subkm_ref_update(_p(X), n, d, k, _p(labels), _p(C), _p(out), _p(cnt))
    return out, shift, cnt


def lloyd(X, C0, max_iter: int, tol: float, trace: bool = False):
    """One Lloyd run. Returns dict(centers, labels, sse, iters[, trace])."""
    X = _f64(X)
    C0 = _f64(C0)
    n, d = X.shape
    k = C0.shape[0]
    C = np.empty_like(C0)
    lab = np.empty(n, np.int32)
    sse = ctypes.c_double()
    tr = np.empty(2 * max_iter + 1, np.float64) if trace else None
    it = _load().subkm_ref_lloyd(_p(X), n, d, k, _p(C0), int(max_iter), float(tol),
                                 _p(C), _p(lab), ctypes.byref(sse), _p(tr))
    if it < 0:
        raise ValueError("invalid arguments")
    out = dict(centers=C, labels=lab, sse=sse.value, iters=int(it))
    if trace:
        out["trace"] = tr
    return out


def local_k(n_r: int, k_local: int, N: int) -> int:
    """Local centers of a subcluster of n_r points: ceil(n_r * k_local / N)."""
    return -(-n_r * k_local // N)


def cluster(X, N: int, k_local: int, k_final: int, max_iter: int, tol: float,
            fixed_landmark: bool = False, scheme: int = 0, m: int = 0, metric: int = 0):
    """The whole two-level method; returns a dict of every intermediate.
    scheme 0 subclusters with Algorithm 1, scheme 1 with Algorithm 2 into m
    groups (0: ceil(n / N))."""
    X = _f32(X)
    n, d = X.shape
    T_cap = -(-n // N) if scheme == 0 or m == 0 else int(m)
    S = np.empty_like(X)
    perm = np.empty(n, np.int64)
    offsets = np.empty(T_cap + 1, np.int64)
    T = ctypes.c_int64()
    M = ctypes.c_int64()
    loc = np.empty((n, d), np.float64)
    lk = np.empty(T_cap, np.int32)
    lit = np.empty(T_cap, np.int32)
    lsse = np.empty(T_cap, np.float64)
    C = np.empty((k_final, d), np.float64)
    lab = np.empty(n, np.int32)
    sse = ctypes.c_double()
    fit = ctypes.c_int32()
    rc = _load().subkm_ref_cluster(_p(X), n, d, int(N), int(k_local), int(k_final), int(max_iter),
                                   float(tol), int(fixed_landmark), int(scheme), int(m),
                                   int(metric),
                                   _p(S), _p(perm), _p(offsets),
                                   ctypes.byref(T), _p(loc), _p(lk), _p(lit), _p(lsse),
                                   ctypes.byref(M), _p(C), _p(lab), ctypes.byref(sse),
                                   ctypes.byref(fit))
    if rc != 0:
        raise ValueError("invalid arguments (code %d)" % rc)
    t = T.value
    return dict(S=S, perm=perm, offsets=offsets[:t + 1].copy(), T=t,
                local_centers=loc[:M.value].copy(), local_k=lk[:t].copy(),
                local_iters=lit[:t].copy(), local_sse=lsse[:t].copy(), M=M.value,
                centers=C, labels=lab, sse=sse.value, final_iters=fit.value)
