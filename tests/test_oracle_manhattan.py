"""Pins of the Manhattan similarity (Sec. II names the Euclidean and the
Manhattan distance as measures of closeness to the landmark) in both
subclustering algorithms of the oracle.

Checked against: hand-worked cases where the two measures disagree,
exhaustive subset enumeration with an independently written L1 key, an
exact rational brute force for Algorithm 2, and the fact that on one
attribute both measures rank every point alike (|x - L| and (x - L)^2 are
both increasing in |x - L|), so the results must coincide there.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import synth


def l1(row, L):
    acc = 0.0
    for a, b in zip(row, L):
        acc = acc + abs(float(a) - float(b))
    return acc


def groups(perm, offsets):
    return [list(perm[offsets[t]:offsets[t + 1]]) for t in range(len(offsets) - 1)]


def test_algorithm1_measures_disagree(oracle):
    # L = (0, 0): A = (3, 0) has L1 3 and squared L2 9; B = (2, 2) has L1 4
    # and squared L2 8.  With N = 2 the first subcluster is {origin, A} under
    # L1 and {origin, B} under L2.
    S = np.array([[3, 0], [2, 2], [0, 0], [5, 5]], np.float32)
    p1, o1, _ = oracle.subcluster(S, 2, metric=1)
    p2, o2, _ = oracle.subcluster(S, 2, metric=0)
    assert groups(p1, o1) == [[0, 2], [1, 3]]
    assert groups(p2, o2) == [[1, 2], [0, 3]]


def test_algorithm1_exhaustive_tiny(oracle):
    rng = np.random.default_rng(17)
    for trial in range(40):
        n = int(rng.integers(1, 10))
        d = int(rng.integers(1, 4))
        N = int(rng.integers(1, n + 1))
        S = rng.integers(0, 5, size=(n, d)).astype(np.float32) / 4  # many ties
        perm, off, L = oracle.subcluster(S, N, metric=1)
        rem = list(range(n))
        for t, g in enumerate(groups(perm, off)):
            Lt = S[rem].min(0)
            np.testing.assert_array_equal(L[t], Lt)
            take = min(N, len(rem))
            ks = {i: (l1(S[i], Lt), i) for i in rem}
            good = [set(c) for c in itertools.combinations(rem, take)
                    if all(ks[a] < ks[b] for a in c for b in rem if b not in c)]
            assert len(good) == 1
            assert set(g) == good[0] and g == sorted(g)
            rem = [i for i in rem if i not in good[0]]
        assert rem == []


def test_algorithm1_fixed_landmark_is_one_sort(oracle):
    S, _, _ = oracle.scale(synth.tiny().X[:2000])
    perm, off, _ = oracle.subcluster(S, 300, fixed_landmark=True, metric=1)
    L = S.min(0).astype(np.float64)
    keys = np.zeros(len(S))
    for j in range(S.shape[1]):  # ascending attributes, as the definition sums
        keys = keys + np.abs(S[:, j].astype(np.float64) - L[j])
    order = np.lexsort((np.arange(len(S)), keys))
    for t in range(len(off) - 1):
        np.testing.assert_array_equal(perm[off[t]:off[t + 1]], np.sort(order[off[t]:off[t + 1]]))


def test_algorithm2_measures_disagree(oracle):
    # L = (0, 0), H = (4, 2), m = 3: landmarks (0,0), (2,1), (4,2).
    # x = (1.375, 0): L1 1.375 to p0 and 1.625 to p1 -> p0; squared L2
    # 1.890625 to p0 and 1.390625 to p1 -> p1.
    S = np.array([[0, 0], [4, 2], [1.375, 0]], np.float32)
    _, o1, _, g1 = oracle.subcluster_unequal(S, 3, metric=1)
    _, o2, _, g2 = oracle.subcluster_unequal(S, 3, metric=0)
    np.testing.assert_array_equal(g1, [0, 2, 0])
    np.testing.assert_array_equal(g2, [0, 2, 1])
    np.testing.assert_array_equal(o1, [0, 2, 2, 3])
    np.testing.assert_array_equal(o2, [0, 1, 2, 3])


def _exact_groups(S, m, metric):
    n, d = S.shape
    L = [Fraction(float(v)) for v in S.min(axis=0)]
    H = [Fraction(float(v)) for v in S.max(axis=0)]
    P = [[L[j] + Fraction(q, max(m - 1, 1)) * (H[j] - L[j]) for j in range(d)] for q in range(m)]
    out, gap = [], []
    for i in range(n):
        x = [Fraction(float(v)) for v in S[i]]
        if metric:
            D = [sum(abs(x[j] - p[j]) for j in range(d)) for p in P]
        else:
            D = [sum((x[j] - p[j]) ** 2 for j in range(d)) for p in P]
        best = min(range(m), key=lambda q: (D[q], q))
        rest = [D[q] for q in range(m) if q != best]
        out.append(best)
        gap.append(float((min(rest) - D[best]) / max(D[best], Fraction(1, 10**30))) if rest else np.inf)
    return np.array(out), np.array(gap)


@pytest.mark.parametrize("m", [2, 6, 11])
def test_algorithm2_exact_rational(oracle, m):
    rng = np.random.default_rng(99 + m)
    S = rng.uniform(-2.0, 3.0, size=(120, 3)).astype(np.float32)
    _, _, _, grp = oracle.subcluster_unequal(S, m, metric=1)
    want, gap = _exact_groups(S, m, 1)
    clear = gap > 1e-9
    assert clear.sum() > 110
    np.testing.assert_array_equal(grp[clear], want[clear])


@pytest.mark.parametrize("alg", [1, 2])
def test_one_attribute_measures_coincide(oracle, alg):
    X = synth.gaussian_blobs(3000, 1, 5, seed=12)[0]
    S, _, _ = oracle.scale(X)
    if alg == 1:
        a = oracle.subcluster(S, 250, metric=0)
        b = oracle.subcluster(S, 250, metric=1)
        np.testing.assert_array_equal(a[0], b[0])
    else:
        a = oracle.subcluster_unequal(S, 17, metric=0)
        b = oracle.subcluster_unequal(S, 17, metric=1)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])


def test_cluster_with_manhattan_keys(oracle):
    # the whole method takes the measure only for subclustering
    job = synth.tiny()
    for scheme in (0, 1):
        r = oracle.cluster(job.X, job.N, job.k_local, job.k_final, 5, 0.0, scheme=scheme, metric=1)
        if scheme == 0:
            perm, off, _ = oracle.subcluster(r["S"], job.N, metric=1)
        else:
            perm, off, _, _ = oracle.subcluster_unequal(r["S"], -(-len(job.X) // job.N), metric=1)
        np.testing.assert_array_equal(r["perm"], perm)
        np.testing.assert_array_equal(r["offsets"], off)


def test_invalid_metric(oracle):
    S = np.zeros((4, 2), np.float32)
    with pytest.raises(ValueError):
        oracle.subcluster(S, 2, metric=2)
    with pytest.raises(ValueError):
        oracle.subcluster_unequal(S, 2, metric=5)
