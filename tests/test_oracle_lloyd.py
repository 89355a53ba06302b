"""Pins of the oracle's Lloyd iteration (the clustering named in Sec. I and
run inside every subcluster, Sec. II Algorithm 1 step 4, and on the local
centers, Sec. V).

Fixed by: exhaustive optimal partitions for n <= 9, the monotone decrease of
the k-means objective, the fixed point at convergence, k=1 (column mean) and
k=n (zero objective), the exact 1-D optimum from dynamic programming, blob
sample means, and library routines for the two steps (argmin of pairwise
distances, group means by bincount).
"""
import itertools

import numpy as np
import pytest
from scipy.spatial.distance import cdist


def sse_of(X, lab, k):
    s = 0.0
    for c in range(k):
        m = X[lab == c]
        if len(m):
            s += float(((m - m.mean(0)) ** 2).sum())
    return s


def test_assign_matches_pairwise_argmin(oracle):
    rng = np.random.default_rng(1)
    X = rng.standard_normal((500, 6))
    C = rng.standard_normal((17, 6))
    lab, sse, dmin, margin = oracle.assign(X, C)
    D = cdist(X, C, "sqeuclidean")
    ok = margin > 1e-9
    np.testing.assert_array_equal(lab[ok], D.argmin(1)[ok])
    np.testing.assert_allclose(dmin, D.min(1), rtol=1e-12)
    np.testing.assert_allclose(sse, D.min(1).sum(), rtol=1e-12)
    Ds = np.sort(D, 1)
    np.testing.assert_allclose(margin, (Ds[:, 1] - Ds[:, 0]) / Ds[:, 1], rtol=1e-9, atol=1e-15)


def test_assign_tie_lowest_index(oracle):
    X = np.array([[0.0, 0.0], [1.0, 1.0]])
    C = np.array([[0.5, 0.5], [0.5, 0.5], [9.0, 9.0]])
    lab, _, _, margin = oracle.assign(X, C)
    np.testing.assert_array_equal(lab, [0, 0])
    np.testing.assert_array_equal(margin, [0.0, 0.0])


def test_update_matches_group_means_and_keeps_empty(oracle):
    rng = np.random.default_rng(2)
    X = rng.standard_normal((300, 5))
    lab = rng.integers(0, 7, 300).astype(np.int32)
    lab[lab == 4] = 5  # center 4 becomes empty
    C = rng.standard_normal((7, 5))
    out, shift, cnt = oracle.update(X, lab, C)
    bc = np.bincount(lab, minlength=7)
    np.testing.assert_array_equal(cnt, bc)
    for c in range(7):
        if bc[c]:
            np.testing.assert_allclose(out[c], X[lab == c].mean(0), rtol=1e-13, atol=1e-15)
        else:
            np.testing.assert_array_equal(out[c], C[c])
    np.testing.assert_allclose(shift, np.linalg.norm(out - C, axis=1).max(), rtol=1e-13)


@pytest.mark.parametrize("seed", range(5))
def test_objective_never_increases(oracle, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((400, 3)) + rng.integers(0, 5, (400, 1))
    r = oracle.lloyd(X, X[:9], 25, 0.0, trace=True)
    tr = r["trace"]
    assert np.all(np.diff(tr) <= 1e-12 * tr[0])
    assert r["sse"] == tr[-1]


def test_fixed_point_at_convergence(oracle):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((300, 4))
    r = oracle.lloyd(X, X[:6], 500, 1e-300)
    assert r["iters"] < 500  # stopped on a zero move
    lab, sse, _, _ = oracle.assign(X, r["centers"])
    np.testing.assert_array_equal(lab, r["labels"])
    out, shift, _ = oracle.update(X, lab, r["centers"])
    assert shift == 0.0
    np.testing.assert_array_equal(out, r["centers"])
    assert sse == r["sse"]


def test_k1_is_column_mean(oracle):
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 1, (123, 7))
    r = oracle.lloyd(X, X[:1], 1, 0.0)
    np.testing.assert_allclose(r["centers"][0], X.mean(0), rtol=1e-14)
    np.testing.assert_allclose(r["sse"], ((X - X.mean(0)) ** 2).sum(), rtol=1e-12)


def test_k_equals_n_gives_zero(oracle):
    rng = np.random.default_rng(5)
    X = rng.uniform(0, 1, (40, 3))
    r = oracle.lloyd(X, X, 3, 0.0)
    assert r["sse"] == 0.0
    np.testing.assert_array_equal(r["labels"], np.arange(40))


def all_partitions_sse(X, k):
    """Optimal k-means objective over every labeling with all k groups used."""
    n = len(X)
    best = np.inf
    for lab in itertools.product(range(k), repeat=n):
        lab = np.array(lab)
        if len(set(lab.tolist())) < k:
            continue
        best = min(best, sse_of(X, lab, k))
    return best


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_optimum(oracle, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(5, 9))
    k = int(rng.integers(2, 4))
    X = rng.uniform(0, 1, (n, 2))
    opt = all_partitions_sse(X, k)
    r = oracle.lloyd(X, X[:k], 50, 0.0)
    assert r["sse"] >= opt - 1e-12
    # started from the optimal partition's centroids, Lloyd stays there
    lab_opt = min((np.array(l) for l in itertools.product(range(k), repeat=n)
                   if len(set(l)) == k), key=lambda l: sse_of(X, l, k))
    C = np.array([X[lab_opt == c].mean(0) for c in range(k)])
    r2 = oracle.lloyd(X, C, 10, 0.0)
    np.testing.assert_allclose(r2["sse"], opt, rtol=1e-12)
    np.testing.assert_allclose(r2["centers"], C, rtol=1e-12, atol=1e-15)


def test_well_separated_reaches_optimum(oracle):
    rng = np.random.default_rng(8)
    centers = np.array([[0, 0], [100, 0], [0, 100]], float)
    grp = np.array([0, 1, 2, 0, 1, 2, 2, 1, 0])
    X = centers[grp] + rng.uniform(-1, 1, (9, 2))
    opt = all_partitions_sse(X, 3)
    r = oracle.lloyd(X, X[:3], 20, 0.0)  # first three points, one per group
    np.testing.assert_allclose(r["sse"], opt, rtol=1e-12)
    np.testing.assert_array_equal(r["labels"], grp)


def ckmeans_1d(x, k):
    """Exact 1-D k-means optimum by dynamic programming over sorted data."""
    x = np.sort(x)
    n = len(x)
    s1 = np.concatenate([[0.0], np.cumsum(x)])
    s2 = np.concatenate([[0.0], np.cumsum(x * x)])

    def cost(i, j):  # points i..j-1
        m = j - i
        return s2[j] - s2[i] - (s1[j] - s1[i]) ** 2 / m

    D = np.full((k + 1, n + 1), np.inf)
    D[0, 0] = 0.0
    for q in range(1, k + 1):
        for j in range(q, n + 1):
            D[q, j] = min(D[q - 1, i] + cost(i, j) for i in range(q - 1, j))
    return D[k, n]


@pytest.mark.parametrize("seed", range(3))
def test_1d_never_below_dp_optimum(oracle, seed):
    rng = np.random.default_rng(200 + seed)
    x = np.concatenate([rng.normal(m, 0.3, 40) for m in (0, 2, 5, 9)])
    rng.shuffle(x)
    X = x[:, None]
    for k in (2, 3, 4, 6):
        r = oracle.lloyd(X, X[:k], 100, 0.0)
        assert r["sse"] >= ckmeans_1d(x, k) * (1 - 1e-12)


def test_blob_means(oracle):
    # one start per blob and no Voronoi leakage: the centers are the blob means
    rng = np.random.default_rng(9)
    mu = np.array([[0, 0, 0], [10, 0, 0], [0, 10, 0], [0, 0, 10]], float)
    grp = np.concatenate([np.arange(4), rng.integers(0, 4, 996)])
    X = mu[grp] + rng.uniform(-1, 1, (1000, 3))
    r = oracle.lloyd(X, X[:4], 5, 0.0)
    for c in range(4):
        np.testing.assert_allclose(r["centers"][c], X[grp == c].mean(0), rtol=1e-13, atol=1e-13)
    np.testing.assert_array_equal(r["labels"], grp)


def test_tolerance_stop_is_strict(oracle):
    X = np.array([[0.0], [2.0], [10.0], [12.0]])
    # start at (0, 2): the first update moves center 1 from 2 to 8 (a move of
    # exactly 6), the second moves it to 11 and center 0 to 1 (moves 3 and 1)
    r = oracle.lloyd(X, X[:2], 10, 6.0)
    assert r["iters"] == 2  # a move of exactly tol does not stop
    r = oracle.lloyd(X, X[:2], 10, 6.0000001)
    assert r["iters"] == 1
    np.testing.assert_array_equal(r["centers"][:, 0], [0.0, 8.0])
