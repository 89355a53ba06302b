"""Pins of the oracle's equal sized subclustering (Sec. II, Algorithm 1).

Checked against: hand-worked examples, exhaustive subset enumeration on tiny
inputs, the partition and nesting properties every correct run must have,
and the reading in which the landmark stays fixed, which reduces the whole
procedure to one global sort (numpy lexsort).
"""
import itertools

import numpy as np
import pytest

import synth


def key(row, L):
    acc = 0.0
    for a, b in zip(row, L):
        q = float(a) - float(b)
        acc = acc + q * q
    return acc


def groups(perm, offsets):
    return [list(perm[offsets[t]:offsets[t + 1]]) for t in range(len(offsets) - 1)]


def test_hand_worked_1d(oracle):
    # d = 1, N = 2.  Round 0: L=0, the two smallest are idx 5 (0.0), idx 1 (0.2).
    # Round 1: remaining {0:1.0, 2:0.6, 3:0.4, 4:0.8}, L = 0.4 -> idx 3, idx 2.
    # Round 2: the rest {0, 4}.
    S = np.array([[1.0], [0.2], [0.6], [0.4], [0.8], [0.0]], np.float32)
    perm, off, L = oracle.subcluster(S, 2)
    assert groups(perm, off) == [[1, 5], [2, 3], [0, 4]]
    np.testing.assert_array_equal(L[:, 0], np.float32([0.0, 0.4, 0.8]))


def test_hand_worked_2d_recomputed_landmark(oracle):
    # N = 1.  With the landmark recomputed over the points left, p1 overtakes
    # p3 in round 2 (L moves to (0.62, 0.1)); with the first landmark kept, the
    # order is the global order of distances to the origin.
    S = np.array([[0.0, 0.0], [1.0, 0.1], [0.1, 0.75], [0.62, 0.62]], np.float32)
    perm, off, L = oracle.subcluster(S, 1)
    assert list(perm) == [0, 2, 1, 3]
    np.testing.assert_array_equal(L[1], np.float32([0.1, 0.1]))
    np.testing.assert_array_equal(L[2], np.float32([0.62, 0.1]))
    permf, _, _ = oracle.subcluster(S, 1, fixed_landmark=True)
    assert list(permf) == [0, 2, 3, 1]


def test_ties_go_to_lower_index(oracle):
    S = np.array([[0.5, 0.5]] * 7, np.float32)
    perm, off, _ = oracle.subcluster(S, 3)
    assert groups(perm, off) == [[0, 1, 2], [3, 4, 5], [6]]


def test_exhaustive_tiny(oracle):
    # every round's subcluster is the unique N-subset of the remaining points
    # whose members all precede all non-members in (key, index) order; find it
    # by enumerating all subsets
    rng = np.random.default_rng(7)
    for trial in range(40):
        n = int(rng.integers(1, 10))
        d = int(rng.integers(1, 4))
        N = int(rng.integers(1, n + 1))
        S = rng.integers(0, 4, size=(n, d)).astype(np.float32) / 4  # many ties
        perm, off, L = oracle.subcluster(S, N)
        rem = list(range(n))
        for t, g in enumerate(groups(perm, off)):
            Lt = S[rem].min(0)
            np.testing.assert_array_equal(L[t], Lt)
            take = min(N, len(rem))
            ks = {i: (key(S[i], Lt), i) for i in rem}
            good = [set(c) for c in itertools.combinations(rem, take)
                    if all(ks[a] < ks[b] for a in c for b in rem if b not in c)]
            assert len(good) == 1
            assert set(g) == good[0] and g == sorted(g)
            rem = [i for i in rem if i not in good[0]]
        assert rem == []


@pytest.mark.parametrize("N", [1, 50, 512, 1000, 4096, 5000])
def test_partition_and_nesting(oracle, N):
    job = synth.tiny()
    S, _, _ = oracle.scale(job.X)
    n = S.shape[0]
    perm, off, L = oracle.subcluster(S, N)
    T = -(-n // N)
    assert len(off) == T + 1 and off[0] == 0 and off[-1] == n
    sizes = np.diff(off)
    assert np.all(sizes[:-1] == N) and 1 <= sizes[-1] <= N
    assert np.array_equal(np.sort(perm), np.arange(n))
    np.testing.assert_array_equal(L[0], 0.0)  # scaled data: the first landmark is the origin
    rem = np.ones(n, bool)
    for t in range(T):
        g = perm[off[t]:off[t + 1]]
        assert np.all(np.diff(g) > 0)
        np.testing.assert_array_equal(L[t], S[rem].min(0))
        rem[g] = False
        if not rem.any():
            break
        # nesting: every member of G_t precedes every later point under L_t
        kg = max((key(S[i], L[t]), i) for i in g)
        rest = np.flatnonzero(rem)
        diff = S[rest].astype(np.float64) - L[t].astype(np.float64)
        kr = np.einsum("ij,ij->i", diff, diff)
        j = np.argmin(kr)
        # the nearest remaining point by a vectorised sum; compare with the exact key
        near = [i for i in rest[np.argsort(kr)[:8]]]
        assert all(kg < (key(S[i], L[t]), i) for i in near)


def test_fixed_landmark_is_one_global_sort(oracle):
    job = synth.tiny()
    S, _, _ = oracle.scale(job.X)
    perm, off, _ = oracle.subcluster(S, 300, fixed_landmark=True)
    L0 = S.min(0).astype(np.float64)
    keys = np.array([key(r, L0) for r in S])
    order = np.lexsort((np.arange(len(S)), keys))
    for t in range(len(off) - 1):
        np.testing.assert_array_equal(perm[off[t]:off[t + 1]], np.sort(order[off[t]:off[t + 1]]))


def test_single_subcluster_identity(oracle):
    S, _, _ = oracle.scale(synth.table1("iris"))
    perm, off, _ = oracle.subcluster(S, 150)
    np.testing.assert_array_equal(perm, np.arange(150))
    np.testing.assert_array_equal(off, [0, 150])
    perm, off, _ = oracle.subcluster(S, 10 ** 6)
    np.testing.assert_array_equal(off, [0, 150])
