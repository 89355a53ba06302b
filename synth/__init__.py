"""Seeded synthetic inputs for subclustered k-means.

This module only draws random numbers and arranges them into the shapes of
the workloads below.  It contains none of the clustering method's arithmetic
(no scaling, no distances, no selection), so both the HIP path and the CPU
oracle can take their inputs from it without sharing any method code.

Every generator is deterministic for a given seed (numpy PCG64 stream).
Labels of mixture components are drawn i.i.d. per point, so the index order
of the points is random and "the first k points of a subcluster" is a random
sample of it.

Workloads (sizes follow the configurations the method is measured on):

* ``tiny``      4096 x 4, 8 isotropic blobs (means U[0,10]^4, sigma 0.5).
* ``mid``       2^20 x 16, 64 blobs, diagonal sigma U[0.2,1.5] per blob and
                attribute, 1% uniform outliers in U[-5,15]^16.
* ``ragged``    512 independent jobs, sizes log-uniform in [1k, 64k], half with
                d=8 and half with d=32, each a mixture of 4..32 components.
* ``precision`` 2^22 x 128, 256 blobs, means N(0, 25 I), sigma 1.
* ``serving``   a Poisson stream of jobs of different n, d and k.
* ``paper2d``   2-D blobs with 500 points per cluster (the timing workload of
                the paper's Sec. VI, Table II).
* ``table1``    150 x 4 and 210 x 7 with 3 blobs (the shapes of the two small
                accuracy datasets of Sec. VI, Table I; synthetic stand-ins).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BASE_SEED = 14121947

# index of each named workload; the default seed of a workload is BASE_SEED + index
WORKLOADS = ("tiny", "mid", "ragged", "precision", "serving")


def default_seed(name: str) -> int:
    return BASE_SEED + WORKLOADS.index(name)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_blobs(n: int, d: int, n_blobs: int, seed: int, *,
                   means: np.ndarray | None = None,
                   mean_low: float = 0.0, mean_high: float = 10.0,
                   sigma: float | tuple[float, float] = 0.5,
                   outlier_frac: float = 0.0,
                   outlier_low: float = -5.0, outlier_high: float = 15.0,
                   chunk: int = 1 << 20):
    """Mixture of Gaussian blobs.

    sigma is either a scalar (isotropic, same for every blob) or a pair
    (lo, hi): then every blob b and attribute j get sigma_bj ~ U[lo, hi]
    (anisotropic diagonal).  An exact count round(outlier_frac * n) of points,
    at seeded indices, is replaced by U[outlier_low, outlier_high]^d.

    Returns (X float32 [n, d] C-contiguous, component label int32 [n], -1 for
    outliers).
    """
    rng = _rng(seed)
    if means is None:
        means = rng.uniform(mean_low, mean_high, size=(n_blobs, d))
    means = np.asarray(means, dtype=np.float64)
    if isinstance(sigma, tuple):
        sig = rng.uniform(sigma[0], sigma[1], size=(n_blobs, d))
    else:
        sig = np.full((n_blobs, d), float(sigma))
    lab = rng.integers(0, n_blobs, size=n, dtype=np.int64)
    X = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        z = rng.standard_normal(size=(e - s, d))
        li = lab[s:e]
        X[s:e] = (means[li] + sig[li] * z).astype(np.float32)
    lab32 = lab.astype(np.int32)
    n_out = int(round(outlier_frac * n))
    if n_out > 0:
        idx = rng.choice(n, size=n_out, replace=False)
        X[idx] = rng.uniform(outlier_low, outlier_high, size=(n_out, d)).astype(np.float32)
        lab32[idx] = -1
    return np.ascontiguousarray(X), lab32


@dataclass(frozen=True)
class ClusterJob:
    """One two-level clustering problem: points plus the method's knobs."""
    X: np.ndarray          # [n, d] float32
    N: int                 # subcluster size
    k_local: int           # centers per full subcluster
    k_final: int           # centers of the final run
    max_iter: int
    tol: float


def tiny(seed: int | None = None) -> ClusterJob:
    seed = default_seed("tiny") if seed is None else seed
    X, _ = gaussian_blobs(4096, 4, 8, seed, sigma=0.5)
    return ClusterJob(X, N=512, k_local=32, k_final=8, max_iter=20, tol=0.0)


def mid(seed: int | None = None, n: int = 1 << 20) -> ClusterJob:
    seed = default_seed("mid") if seed is None else seed
    X, _ = gaussian_blobs(n, 16, 64, seed, sigma=(0.2, 1.5), outlier_frac=0.01)
    return ClusterJob(X, N=8192, k_local=256, k_final=64, max_iter=30, tol=1e-6)


def precision(seed: int | None = None, n: int = 1 << 22) -> ClusterJob:
    seed = default_seed("precision") if seed is None else seed
    rng = _rng(seed + 1000)
    means = rng.normal(0.0, 5.0, size=(256, 128))
    X, _ = gaussian_blobs(n, 128, 256, seed, means=means, sigma=1.0)
    return ClusterJob(X, N=32768, k_local=1024, k_final=256, max_iter=30, tol=1e-6)


@dataclass(frozen=True)
class RaggedSet:
    """Independent Lloyd runs of different sizes and dimensionalities."""
    X: list            # list of float32 [n_j, d_j]
    k: list            # centers per run
    max_iter: int
    tol: float


def ragged(seed: int | None = None, runs: int = 512, lo: int = 1024, hi: int = 65536,
           dims=(8, 32), k_cap: int = 1024, compression: int = 32) -> RaggedSet:
    """Sizes log-uniform in [lo, hi], exactly half the runs at each d (seeded
    shuffle), k_j = min(ceil(n_j / compression), k_cap), each run a mixture
    of U{4..32} components with means U[0,10]^d and sigma U[0.2,1.5]."""
    seed = default_seed("ragged") if seed is None else seed
    rng = _rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=runs))).astype(np.int64)
    ds = np.array([dims[i * len(dims) // runs] for i in range(runs)])
    rng.shuffle(ds)
    Xs, ks = [], []
    for j in range(runs):
        m = int(rng.integers(4, 33))
        sub = int(rng.integers(0, 2**62))
        X, _ = gaussian_blobs(int(sizes[j]), int(ds[j]), m, sub, sigma=(0.2, 1.5))
        Xs.append(X)
        ks.append(int(min(-(-int(sizes[j]) // compression), k_cap)))
    return RaggedSet(Xs, ks, max_iter=30, tol=1e-6)


@dataclass(frozen=True)
class ServeRequest:
    arrival_s: float
    n: int
    d: int
    k_final: int
    seed: int


def serving_stream(jobs: int, rate_hz: float = 50.0, seed: int | None = None,
                   n_lo: int = 10_000, n_hi: int = 2_000_000,
                   dims=(4, 8, 16, 32, 64), k_lo: int = 8, k_hi: int = 256):
    """Poisson arrivals; n log-uniform in [n_lo, n_hi], d uniform in dims,
    final k uniform in [k_lo, k_hi].  Points are drawn lazily with
    :func:`serving_points` from the per-job seed."""
    seed = default_seed("serving") if seed is None else seed
    rng = _rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=jobs))
    ns = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=jobs))).astype(np.int64)
    ds = rng.choice(np.array(dims), size=jobs)
    ks = rng.integers(k_lo, k_hi + 1, size=jobs)
    seeds = rng.integers(0, 2**62, size=jobs)
    return [ServeRequest(float(t[i]), int(ns[i]), int(ds[i]), int(ks[i]), int(seeds[i]))
            for i in range(jobs)]


def serving_points(req: ServeRequest) -> np.ndarray:
    X, _ = gaussian_blobs(req.n, req.d, req.k_final, req.seed, sigma=0.5)
    return X


def serving_pool(dims=(4, 8, 16, 32, 64), n_max: int = 2_000_000, blobs: int = 128,
                 seed: int | None = None) -> dict:
    """One point pool per attribute count for a served stream: n_max points
    of `blobs` Gaussian blobs (means U[0,10]^d, sigma 0.5).  A job of n points
    takes n consecutive rows at a seeded offset (see :func:`pool_slice`), so
    a long stream needs no per-job generation."""
    seed = default_seed("serving") if seed is None else seed
    return {d: gaussian_blobs(n_max, d, blobs, seed + 17 * d, sigma=0.5)[0] for d in dims}


def pool_slice(req: ServeRequest, n_max: int) -> tuple:
    """(first row, n) of a request's points inside its pool."""
    off = int(np.random.default_rng(req.seed).integers(0, n_max - req.n + 1))
    return off, req.n


def paper2d(n: int, seed: int = BASE_SEED + 100, per_cluster: int = 500) -> np.ndarray:
    """2-D blobs with ``per_cluster`` points per cluster on average."""
    k = max(1, n // per_cluster)
    X, _ = gaussian_blobs(n, 2, k, seed, mean_low=0.0, mean_high=100.0, sigma=0.5)
    return X


def table1(which: str, seed: int = BASE_SEED + 200) -> np.ndarray:
    """150 x 4 or 210 x 7 with three blobs (shape stand-ins only)."""
    n, d = {"iris": (150, 4), "seeds": (210, 7)}[which]
    X, _ = gaussian_blobs(n, d, 3, seed, mean_low=0.0, mean_high=6.0, sigma=0.6)
    return X
