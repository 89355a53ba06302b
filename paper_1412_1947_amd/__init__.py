"""Python binding of libsubkm (include/subkm.h): subclustered k-means on
AMD Instinct MI355X.

Argument marshalling only.  Every step of the method runs in the HIP
library; PyTorch supplies device memory and the stream.  There is no CPU
fallback: without the built library (``__graft_entry__.build()``) or without
a GPU every call raises.

The method (arXiv 1412.1947): min-max feature scaling, equal sized
subclustering (Sec. II, Algorithm 1) or unequal sized subclustering (Sec.
III, Algorithm 2), Lloyd's k-means inside every subcluster and on the local
centers (Sec. I, Sec. V).
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import threading
import weakref

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsubkm.so")

PREC_FP32 = 0
PREC_BF16 = 1
FORM_BATCHED = 0
FORM_PLAIN = 1
SCHEME_EQUAL = 0    # Algorithm 1
SCHEME_UNEQUAL = 1  # Algorithm 2
METRIC_L2 = 0       # squared Euclidean similarity to the landmark
METRIC_L1 = 1       # Manhattan similarity to the landmark
LAYOUT_ROW = 0      # X is n x d, row-major
LAYOUT_COL = 1      # X is d x n (column-major points)


class SubkmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libsubkm status {status}: {msg}")
        self.status = status


class Run(ctypes.Structure):
    _fields_ = [("x_off", ctypes.c_int64), ("n", ctypes.c_int64), ("c_off", ctypes.c_int64),
                ("lab_off", ctypes.c_int64), ("d", ctypes.c_int32), ("k", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("landmark_mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("form", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("S", ctypes.c_void_p), ("perm", ctypes.c_void_p),
                ("local_centers", ctypes.c_void_p), ("local_iters", ctypes.c_void_p),
                ("local_sse", ctypes.c_void_p), ("m", ctypes.c_int64),
                ("metric", ctypes.c_int32), ("layout", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int64), ("M", ctypes.c_int64), ("final_iters", ctypes.c_int32),
                ("sub_selections", ctypes.c_int32), ("local_point_iters", ctypes.c_int64),
                ("final_point_iters", ctypes.c_int64), ("us_scale", ctypes.c_double),
                ("us_subcluster", ctypes.c_double), ("us_local", ctypes.c_double),
                ("us_final", ctypes.c_double), ("us_label", ctypes.c_double),
                ("us_total", ctypes.c_double), ("rechecked", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class Job(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("n", ctypes.c_int64), ("N", ctypes.c_int64),
                ("d", ctypes.c_int32), ("k_local", ctypes.c_int32), ("k_final", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("precision", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("centers", ctypes.c_void_p), ("labels", ctypes.c_void_p)]


class JobResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slot", ctypes.c_int32), ("sse", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("footprint", ctypes.c_size_t), ("device_bytes", ctypes.c_size_t),
                ("slot_bytes_admitted", ctypes.c_size_t), ("slot_bytes_after", ctypes.c_size_t),
                ("message", ctypes.c_char * 128)]


EXPORTS = ("subkm_create", "subkm_destroy", "subkm_last_error", "subkm_set_stream",
           "subkm_synchronize", "subkm_scale", "subkm_scale_noalloc", "subkm_scale_colmajor",
           "subkm_subcluster",
           "subkm_subcluster_unequal",
           "subkm_lloyd_batched",
           "subkm_cluster", "subkm_cluster_sizes", "subkm_cluster_footprint", "subkm_device_bytes",
           "subkm_profile_enable", "subkm_profile_query", "subkm_profile_name",
           "subkm_engine_create", "subkm_engine_destroy", "subkm_engine_last_error",
           "subkm_job_footprint", "subkm_engine_submit", "subkm_engine_poll", "subkm_engine_wait",
           "subkm_engine_stats", "subkm_tune_enable", "subkm_tune_count", "subkm_tune_save",
           "subkm_tune_load")

KERNEL_CLASSES = ("assign", "update", "keys", "cand", "scatter", "scale", "lloyd_fused",
                  "subcluster")

_lib = None
_lib_lock = threading.Lock()


def lib():
    """The loaded libsubkm (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
            L = ctypes.CDLL(LIB_PATH)
            P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
            st = ctypes.c_int
            L.subkm_create.argtypes = [ctypes.c_int, P, ctypes.POINTER(P)]
            L.subkm_create.restype = st
            L.subkm_destroy.argtypes = [P]
            L.subkm_destroy.restype = None
            L.subkm_last_error.argtypes = [P]
            L.subkm_last_error.restype = ctypes.c_char_p
            L.subkm_set_stream.argtypes = [P, P]
            L.subkm_set_stream.restype = st
            L.subkm_synchronize.argtypes = [P]
            L.subkm_synchronize.restype = st
            L.subkm_scale.argtypes = [P, P, i64, i32, P, P, P]
            L.subkm_scale.restype = st
            L.subkm_scale_noalloc.argtypes = [P, P, i64, i32, P, P, P]
            L.subkm_scale_noalloc.restype = st
            L.subkm_scale_colmajor.argtypes = [P, P, i64, i32, P, P, P]
            L.subkm_scale_colmajor.restype = st
            L.subkm_subcluster.argtypes = [P, P, i64, i32, i64, i32, i32, P, P, P, P]
            L.subkm_subcluster.restype = st
            L.subkm_subcluster_unequal.argtypes = [P, P, i64, i32, i64, i32, P, P, P, P]
            L.subkm_subcluster_unequal.restype = st
            L.subkm_lloyd_batched.argtypes = [P, P, ctypes.POINTER(Run), i32, P, P, i32, f64, i32,
                                              i32, P, P]
            L.subkm_lloyd_batched.restype = st
            L.subkm_cluster.argtypes = [P, P, i64, i32, i64, i32, i32, i32, f64,
                                        ctypes.POINTER(Opts), P, P, P, ctypes.POINTER(Stats)]
            L.subkm_cluster.restype = st
            L.subkm_cluster_sizes.argtypes = [i64, i64, i32, ctypes.POINTER(i64), ctypes.POINTER(i64)]
            L.subkm_cluster_sizes.restype = st
            L.subkm_cluster_footprint.argtypes = [i64, i32, i64, i32, i32]
            L.subkm_cluster_footprint.restype = ctypes.c_size_t
            L.subkm_device_bytes.argtypes = [P]
            L.subkm_device_bytes.restype = ctypes.c_size_t
            L.subkm_engine_create.argtypes = [ctypes.c_int, ctypes.c_size_t, i32, ctypes.POINTER(P)]
            L.subkm_engine_create.restype = st
            L.subkm_engine_destroy.argtypes = [P]
            L.subkm_engine_destroy.restype = None
            L.subkm_engine_last_error.argtypes = [P]
            L.subkm_engine_last_error.restype = ctypes.c_char_p
            L.subkm_job_footprint.argtypes = [ctypes.POINTER(Job)]
            L.subkm_job_footprint.restype = ctypes.c_size_t
            L.subkm_engine_submit.argtypes = [P, ctypes.POINTER(Job), ctypes.POINTER(i64)]
            L.subkm_engine_submit.restype = st
            L.subkm_engine_poll.argtypes = [P, i64, ctypes.POINTER(i32), ctypes.POINTER(JobResult)]
            L.subkm_engine_poll.restype = st
            L.subkm_engine_wait.argtypes = [P, i64, ctypes.POINTER(JobResult)]
            L.subkm_engine_wait.restype = st
            L.subkm_engine_stats.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                             ctypes.POINTER(ctypes.c_size_t)]
            L.subkm_engine_stats.restype = st
            L.subkm_tune_enable.argtypes = [P, i32]
            L.subkm_tune_enable.restype = st
            L.subkm_tune_count.argtypes = [P, ctypes.POINTER(i32)]
            L.subkm_tune_count.restype = st
            L.subkm_tune_save.argtypes = [P, ctypes.c_char_p]
            L.subkm_tune_save.restype = st
            L.subkm_tune_load.argtypes = [P, ctypes.c_char_p]
            L.subkm_tune_load.restype = st
            L.subkm_profile_enable.argtypes = [P, i32]
            L.subkm_profile_enable.restype = st
            L.subkm_profile_query.argtypes = [P, i32, ctypes.POINTER(i64), ctypes.POINTER(f64)]
            L.subkm_profile_query.restype = st
            L.subkm_profile_name.argtypes = [i32]
            L.subkm_profile_name.restype = ctypes.c_char_p
            _lib = L
    return _lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def cluster_sizes(n: int, N: int, k_local: int):
    T, M = ctypes.c_int64(), ctypes.c_int64()
    st = lib().subkm_cluster_sizes(n, N, k_local, ctypes.byref(T), ctypes.byref(M))
    if st != 0:
        raise SubkmError(st, "invalid sizes")
    return T.value, M.value


def cluster_footprint(n: int, d: int, N: int, k_local: int, k_final: int) -> int:
    return int(lib().subkm_cluster_footprint(n, d, N, k_local, k_final))


class Context:
    """A libsubkm context on one GPU; calls run on torch's current stream."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("libsubkm needs a ROCm GPU; none is visible")
        self.device = int(device)
        h = ctypes.c_void_p()
        st = lib().subkm_create(self.device, None, ctypes.byref(h))
        if st != 0:
            raise SubkmError(st, lib().subkm_last_error(None).decode())
        self._h = h
        _live_handles.add(self)

    def close(self):
        if getattr(self, "_h", None):
            lib().subkm_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # during interpreter shutdown the HIP runtime (and a profiler
        # attached to it) may already be torn down: contexts still open then
        # were closed by the exit handler below, or are left to the process
        # exit (the check is bound at definition: module globals may already
        # be cleared when this runs)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -------------------------------------------------------------
    def _check(self, st):
        if st != 0:
            raise SubkmError(st, lib().subkm_last_error(self._h).decode())

    def _bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self._check(lib().subkm_set_stream(self._h, ctypes.c_void_p(s)))

    def _dev(self, t, dtype, name):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.device.index != self.device:
            raise ValueError(f"{name} must be a tensor on cuda:{self.device}")
        if t.dtype != dtype or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} tensor")
        return t

    def _empty(self, shape, dtype):
        return torch.empty(shape, dtype=dtype, device=f"cuda:{self.device}")

    def synchronize(self):
        self._check(lib().subkm_synchronize(self._h))

    def device_bytes(self) -> int:
        """Device memory the context holds as scratch."""
        return int(lib().subkm_device_bytes(self._h))

    def tune(self, on: bool = True):
        """Schedule tuner of the batched form (results do not depend on it)."""
        self._check(lib().subkm_tune_enable(self._h, 1 if on else 0))

    def tuned(self) -> int:
        """Number of shapes with a tuned schedule."""
        n = ctypes.c_int32()
        self._check(lib().subkm_tune_count(self._h, ctypes.byref(n)))
        return n.value

    def tune_save(self, path: str):
        self._check(lib().subkm_tune_save(self._h, os.fsencode(path)))

    def tune_load(self, path: str):
        self._check(lib().subkm_tune_load(self._h, os.fsencode(path)))

    def profile(self, on: bool = True):
        """Start (or stop) per-launch kernel timing; resets the counters."""
        self._check(lib().subkm_profile_enable(self._h, int(bool(on))))

    def profile_read(self):
        """{class: (launches, total ms)} of the launches timed so far."""
        out = {}
        for c, name in enumerate(KERNEL_CLASSES):
            n, ms = ctypes.c_int64(), ctypes.c_double()
            self._check(lib().subkm_profile_query(self._h, c, ctypes.byref(n), ctypes.byref(ms)))
            out[name] = (n.value, ms.value)
        return out

    # -- the C ABI -------------------------------------------------------------
    def scale(self, X, out=None, layout: int = LAYOUT_ROW):
        """Min-max scaling. X is n x d (LAYOUT_ROW) or d x n (LAYOUT_COL, the
        column-major layout of the points); S is n x d either way.  Returns
        (S, mins, maxs)."""
        X = self._dev(X, torch.float32, "X")
        if layout == LAYOUT_COL:
            d, n = X.shape
        else:
            n, d = X.shape
        S = self._empty((n, d), torch.float32) if out is None else self._dev(out, torch.float32, "out")
        mins = self._empty((d,), torch.float32)
        maxs = self._empty((d,), torch.float32)
        self._bind_stream()
        fn = lib().subkm_scale_colmajor if layout == LAYOUT_COL else lib().subkm_scale
        self._check(fn(self._h, _ptr(X), n, d, _ptr(S), _ptr(mins), _ptr(maxs)))
        return S, mins, maxs

    def scale_noalloc(self, X, S, mins, maxs):
        """Min-max scaling through the allocation-free entry point: the
        caller passes every output (S n x d, mins and maxs d, float32)."""
        X = self._dev(X, torch.float32, "X")
        n, d = X.shape
        S = self._dev(S, torch.float32, "S")
        mins = self._dev(mins, torch.float32, "mins")
        maxs = self._dev(maxs, torch.float32, "maxs")
        if tuple(S.shape) != (n, d) or mins.numel() != d or maxs.numel() != d:
            raise ValueError("S must be n x d and mins, maxs of d values")
        self._bind_stream()
        self._check(lib().subkm_scale_noalloc(self._h, _ptr(X), n, d, _ptr(S), _ptr(mins), _ptr(maxs)))
        return S, mins, maxs

    def subcluster(self, S, N: int, landmark_mode: int = 0, landmarks: bool = False,
                   metric: int = METRIC_L2):
        """Algorithm 1. Returns (P, perm, offsets[, landmarks])."""
        S = self._dev(S, torch.float32, "S")
        n, d = S.shape
        T = -(-n // int(N)) if N >= 1 else 0
        P = self._empty((n, d), torch.float32)
        perm = self._empty((n,), torch.int32)
        offs = self._empty((T + 1,), torch.int64)
        lm = self._empty((T, d), torch.float32) if landmarks else None
        self._bind_stream()
        self._check(lib().subkm_subcluster(self._h, _ptr(S), n, d, int(N), int(landmark_mode),
                                           int(metric), _ptr(P), _ptr(perm), _ptr(offs), _ptr(lm)))
        return (P, perm, offs, lm) if landmarks else (P, perm, offs)

    def subcluster_unequal(self, S, m: int, landmarks: bool = False, metric: int = METRIC_L2):
        """Algorithm 2 into m groups. Returns (P, perm, offsets[, landmarks])."""
        S = self._dev(S, torch.float32, "S")
        n, d = S.shape
        m = int(m)
        P = self._empty((n, d), torch.float32)
        perm = self._empty((n,), torch.int32)
        offs = self._empty((max(m, 0) + 1,), torch.int64)
        lm = self._empty((max(m, 0), d), torch.float64) if landmarks else None
        self._bind_stream()
        self._check(lib().subkm_subcluster_unequal(self._h, _ptr(S), n, d, m, int(metric), _ptr(P),
                                                   _ptr(perm), _ptr(offs), _ptr(lm)))
        return (P, perm, offs, lm) if landmarks else (P, perm, offs)

    def lloyd_batched(self, P, runs, C, labels, max_iter: int, tol: float,
                      precision: int = PREC_FP32, form: int = FORM_BATCHED):
        """Lloyd runs described by `runs` (tuples x_off, n, c_off, lab_off, d, k).
        C holds the starting centers and receives the result.  Returns (iters, sse)."""
        P = self._dev(P, torch.float32, "P")
        C = self._dev(C, torch.float32, "C")
        labels = self._dev(labels, torch.int32, "labels")
        R = len(runs)
        arr = (Run * max(R, 1))(*[Run(*map(int, r)) for r in runs])
        iters = self._empty((max(R, 1),), torch.int32)
        sse = self._empty((max(R, 1),), torch.float64)
        self._bind_stream()
        self._check(lib().subkm_lloyd_batched(self._h, _ptr(P), arr, R, _ptr(C), _ptr(labels),
                                              int(max_iter), float(tol), int(precision), int(form),
                                              _ptr(iters), _ptr(sse)))
        return iters[:R], sse[:R]

    def cluster(self, X, N: int, k_local: int, k_final: int, max_iter: int, tol: float,
                landmark_mode: int = 0, precision: int = PREC_FP32, form: int = FORM_BATCHED,
                intermediates: bool = False, stats: bool = False, scheme: int = SCHEME_EQUAL,
                m: int = 0, metric: int = METRIC_L2, layout: int = LAYOUT_ROW):
        """The whole two-level method (scheme SCHEME_EQUAL: Algorithm 1;
        SCHEME_UNEQUAL: Algorithm 2 into m groups, 0 for ceil(n / N)).  Returns
        a dict with centers (scaled space), labels, sse and, on request,
        intermediates and phase stats.  With Algorithm 2, local_centers holds
        room for the largest possible M; stats["M"] rows of it are used."""
        X = self._dev(X, torch.float32, "X")
        if layout == LAYOUT_COL:
            d, n = X.shape
        else:
            n, d = X.shape
        out = {}
        o = Opts(landmark_mode=int(landmark_mode), precision=int(precision), form=int(form),
                 scheme=int(scheme), m=int(m), metric=int(metric), layout=int(layout))
        if intermediates:
            T, M = cluster_sizes(n, int(N), int(k_local))
            if scheme == SCHEME_UNEQUAL:
                T = int(m) if m else T
                M = min(n, n * int(k_local) // int(N) + T)
            out["S"] = self._empty((n, d), torch.float32)
            out["perm"] = self._empty((n,), torch.int32)
            out["local_centers"] = self._empty((M, d), torch.float32)
            out["local_iters"] = self._empty((T,), torch.int32)
            out["local_sse"] = self._empty((T,), torch.float64)
            o.S, o.perm = out["S"].data_ptr(), out["perm"].data_ptr()
            o.local_centers = out["local_centers"].data_ptr()
            o.local_iters = out["local_iters"].data_ptr()
            o.local_sse = out["local_sse"].data_ptr()
        centers = self._empty((k_final, d), torch.float32)
        labels = self._empty((n,), torch.int32)
        sse = self._empty((1,), torch.float64)
        st = Stats() if stats else None
        self._bind_stream()
        self._check(lib().subkm_cluster(self._h, _ptr(X), n, d, int(N), int(k_local), int(k_final),
                                        int(max_iter), float(tol), ctypes.byref(o), _ptr(centers),
                                        _ptr(labels), _ptr(sse),
                                        ctypes.byref(st) if st is not None else None))
        out.update(centers=centers, labels=labels, sse=sse)
        if st is not None:
            out["stats"] = st.as_dict()
        return out


_contexts: dict = {}
# every open context and engine, closed at interpreter exit while the HIP
# runtime is still whole (engines first: they own contexts of their own)
_live_handles: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_all():
    live = list(_live_handles)
    for h in [x for x in live if isinstance(x, Engine)] + [x for x in live if isinstance(x, Context)]:
        try:
            h.close()
        except Exception:
            pass
    _contexts.clear()


def context(device: int = 0) -> Context:
    """The shared context of a device (created on first use)."""
    c = _contexts.get(device)
    if c is None:
        c = _contexts[device] = Context(device)
    return c


def scale(X, layout=LAYOUT_ROW):
    return context(X.device.index or 0).scale(X, layout=layout)


def subcluster(S, N, landmark_mode=0, landmarks=False, metric=METRIC_L2):
    return context(S.device.index or 0).subcluster(S, N, landmark_mode, landmarks, metric)


def subcluster_unequal(S, m, landmarks=False, metric=METRIC_L2):
    return context(S.device.index or 0).subcluster_unequal(S, m, landmarks, metric)


def lloyd_batched(P, runs, C, labels, max_iter, tol, precision=PREC_FP32, form=FORM_BATCHED):
    return context(P.device.index or 0).lloyd_batched(P, runs, C, labels, max_iter, tol,
                                                      precision, form)


def cluster(X, N, k_local, k_final, max_iter, tol, **kw):
    return context(X.device.index or 0).cluster(X, N, k_local, k_final, max_iter, tol, **kw)


class Engine:
    """Serving engine on one GPU (subkm_engine_*): whole clustering jobs
    submitted from host memory, admitted in arrival order as slots and the
    device memory budget allow, run concurrently on separate streams.

    Inputs are CPU float32 tensors [n, d] (pinned memory lets the copies
    overlap other jobs); results come back in pinned CPU tensors."""

    def __init__(self, device: int = 0, budget_bytes: int = 200 << 30, slots: int = 4):
        h = ctypes.c_void_p()
        st = lib().subkm_engine_create(device, int(budget_bytes), int(slots), ctypes.byref(h))
        if st != 0:
            raise SubkmError(st, "engine creation failed")
        self._h = h
        self._live = {}
        self._lock = threading.Lock()
        _live_handles.add(self)

    def close(self):
        if getattr(self, "_h", None):
            lib().subkm_engine_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def submit(self, X, N: int, k_local: int, k_final: int, max_iter: int, tol: float,
               precision: int = PREC_FP32, labels: bool = True) -> int:
        if X.device.type != "cpu" or X.dtype != torch.float32 or X.dim() != 2:
            raise ValueError("X must be a 2-D float32 CPU tensor")
        X = X.contiguous()
        n, d = X.shape
        cen = torch.empty((k_final, d), dtype=torch.float32, pin_memory=True)
        lab = torch.empty((n,), dtype=torch.int32, pin_memory=True) if labels else None
        job = Job(X.data_ptr(), n, int(N), d, int(k_local), int(k_final), int(max_iter), float(tol),
                  int(precision), 0, cen.data_ptr(), lab.data_ptr() if lab is not None else None)
        jid = ctypes.c_int64()
        st = lib().subkm_engine_submit(self._h, ctypes.byref(job), ctypes.byref(jid))
        if st != 0:
            raise SubkmError(st, lib().subkm_engine_last_error(self._h).decode())
        with self._lock:
            self._live[jid.value] = (X, cen, lab)
        return jid.value

    def _result(self, jid, r: JobResult):
        with self._lock:
            X, cen, lab = self._live.pop(jid)
        if r.status != 0:
            raise SubkmError(r.status, r.message.decode())
        return {"centers": cen, "labels": lab, "sse": r.sse, "slot": r.slot,
                "t_submit": r.t_submit, "t_admit": r.t_admit, "t_start": r.t_start,
                "t_done": r.t_done, "footprint": r.footprint, "device_bytes": r.device_bytes,
                "slot_bytes_admitted": r.slot_bytes_admitted, "slot_bytes_after": r.slot_bytes_after}

    def wait(self, jid: int):
        r = JobResult()
        st = lib().subkm_engine_wait(self._h, jid, ctypes.byref(r))
        if st != 0:
            raise SubkmError(st, "unknown job")
        return self._result(jid, r)

    def poll(self, jid: int):
        r = JobResult()
        done = ctypes.c_int32()
        st = lib().subkm_engine_poll(self._h, jid, ctypes.byref(done), ctypes.byref(r))
        if st != 0:
            raise SubkmError(st, "unknown job")
        return self._result(jid, r) if done.value else None

    def stats(self):
        q, r, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
        lib().subkm_engine_stats(self._h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(b))
        return {"queued": q.value, "running": r.value, "device_bytes": b.value}


def job_footprint(n: int, d: int, N: int, k_local: int, k_final: int) -> int:
    job = Job(None, n, N, d, k_local, k_final, 0, 0.0, 0, 0, None, None)
    return int(lib().subkm_job_footprint(ctypes.byref(job)))
