"""Pins of the oracle's unequal sized subclustering (Sec. III, Algorithm 2).

The landmarks lie evenly on the segment between the attribute-wise minimum L
and maximum H of the points, both ends included; every point joins its
nearest landmark (the lower landmark on a tie) and the groups are kept in
landmark order with ascending indices.  The pins below check the oracle
against hand-worked cases, an exact rational computation, the closed form
that holds for min-max scaled data (the nearest landmark is the one whose
position on the segment is nearest the mean attribute), and the structural
facts of the partition.
"""
from fractions import Fraction

import numpy as np
import pytest

import synth


def test_hand_worked_1d_with_ties(oracle):
    # landmarks 0, 0.5, 1; 0.25 and 0.75 lie halfway between two of them
    S = np.array([[0.0], [0.25], [0.75], [1.0], [0.5]], np.float32)
    perm, offs, lms, grp = oracle.subcluster_unequal(S, 3)
    np.testing.assert_array_equal(lms[:, 0], [0.0, 0.5, 1.0])
    np.testing.assert_array_equal(grp, [0, 0, 1, 2, 1])
    np.testing.assert_array_equal(perm, [0, 1, 2, 4, 3])
    np.testing.assert_array_equal(offs, [0, 2, 4, 5])


def test_hand_worked_2d(oracle):
    # L = (0, 0), H = (2, 4); landmarks (0,0), (1,2), (2,4).
    # (2,0): 4 / 5 / 16 -> 0;  (0,4): 16 / 5 / 4 -> 2
    S = np.array([[0, 0], [2, 4], [1, 2], [2, 0], [0, 4]], np.float32)
    perm, offs, lms, grp = oracle.subcluster_unequal(S, 3)
    np.testing.assert_array_equal(lms, [[0, 0], [1, 2], [2, 4]])
    np.testing.assert_array_equal(grp, [0, 2, 1, 0, 2])
    np.testing.assert_array_equal(perm, [0, 3, 2, 1, 4])
    np.testing.assert_array_equal(offs, [0, 2, 3, 5])


def _exact_groups(S, m):
    """Nearest landmark of every point in exact rational arithmetic, with the
    relative gap between the two smallest squared distances."""
    n, d = S.shape
    L = [Fraction(float(v)) for v in S.min(axis=0)]
    H = [Fraction(float(v)) for v in S.max(axis=0)]
    P = [[L[j] + Fraction(q, max(m - 1, 1)) * (H[j] - L[j]) for j in range(d)]
         for q in range(m)]
    out, gap = [], []
    for i in range(n):
        x = [Fraction(float(v)) for v in S[i]]
        D = [sum((x[j] - p[j]) ** 2 for j in range(d)) for p in P]
        best = min(range(m), key=lambda q: (D[q], q))
        rest = [D[q] for q in range(m) if q != best]
        out.append(best)
        gap.append(float((min(rest) - D[best]) / max(D[best], Fraction(1, 10**30)))
                   if rest else np.inf)
    return np.array(out), np.array(gap)


@pytest.mark.parametrize("m", [2, 5, 9])
def test_exact_rational_brute_force(oracle, m):
    rng = np.random.default_rng(1412 + m)
    S = rng.uniform(-3.0, 5.0, size=(120, 3)).astype(np.float32)
    _, _, lms, grp = oracle.subcluster_unequal(S, m)
    want, gap = _exact_groups(S, m)
    clear = gap > 1e-9  # outside the reach of binary64 rounding
    assert clear.sum() > 110
    np.testing.assert_array_equal(grp[clear], want[clear])
    # the binary64 landmarks are the rational ones to within rounding
    L, H = S.min(axis=0).astype(np.float64), S.max(axis=0).astype(np.float64)
    for q in range(m):
        np.testing.assert_allclose(lms[q], L + q / (m - 1) * (H - L), rtol=0, atol=1e-14)
    np.testing.assert_array_equal(lms[0], L)
    np.testing.assert_array_equal(lms[-1], H)


@pytest.mark.parametrize("m", [3, 16, 41])
def test_closed_form_on_scaled_data(oracle, m):
    # After min-max scaling L = 0 and H = 1 in every attribute, so p_q is the
    # constant q/(m-1) and ||x - p_q||^2 = ||x||^2 - 2 d t_q mean(x) + d t_q^2:
    # the nearest landmark is the one with t_q nearest mean(x).
    X = synth.gaussian_blobs(3000, 6, 7, seed=31 + m)[0]
    S, _, _ = oracle.scale(X)
    _, _, lms, grp = oracle.subcluster_unequal(S, m)
    np.testing.assert_array_equal(lms, np.repeat((np.arange(m) / (m - 1))[:, None], 6, axis=1))
    u = S.astype(np.float64).mean(axis=1) * (m - 1)
    clear = np.abs(u - np.floor(u) - 0.5) > 1e-6
    assert clear.mean() > 0.99
    np.testing.assert_array_equal(grp[clear], np.floor(u[clear] + 0.5).astype(np.int32))


def _check_partition(perm, offs, grp, n, m):
    assert len(offs) == m + 1 and offs[0] == 0 and offs[-1] == n
    assert np.all(np.diff(offs) >= 0)
    np.testing.assert_array_equal(np.sort(perm), np.arange(n))
    np.testing.assert_array_equal(np.diff(offs), np.bincount(grp, minlength=m))
    for q in range(m):
        mem = perm[offs[q]:offs[q + 1]]
        assert np.all(np.diff(mem) > 0)
        assert np.all(grp[mem] == q)


@pytest.mark.parametrize("m", [1, 2, 7, 64, 700])
def test_partition_and_nearest(oracle, m):
    X = synth.gaussian_blobs(600, 5, 9, seed=77)[0]
    S, _, _ = oracle.scale(X)
    perm, offs, lms, grp = oracle.subcluster_unequal(S, m)
    _check_partition(perm, offs, grp, len(S), m)
    # nearest landmark by an independent distance matrix, where the two
    # smallest distances are clearly apart
    D = ((S.astype(np.float64)[:, None, :] - lms[None, :, :]) ** 2).sum(axis=2)
    srt = np.sort(D, axis=1)
    clear = (srt[:, 1] - srt[:, 0] > 1e-12 * (1 + srt[:, 0])) if m > 1 else np.ones(len(S), bool)
    np.testing.assert_array_equal(grp[clear], D.argmin(axis=1)[clear])


def test_single_landmark_is_identity(oracle):
    S = synth.gaussian_blobs(257, 4, 3, seed=5)[0]
    perm, offs, lms, grp = oracle.subcluster_unequal(S, 1)
    np.testing.assert_array_equal(perm, np.arange(257))
    np.testing.assert_array_equal(offs, [0, 257])
    np.testing.assert_array_equal(lms[0], S.min(axis=0))
    assert np.all(grp == 0)


def test_constant_attribute_changes_nothing(oracle):
    # a constant attribute has L_j = H_j, so every landmark equals it there
    S = synth.gaussian_blobs(500, 3, 4, seed=8)[0]
    Sc = np.concatenate([S[:, :1], np.full((500, 1), 0.3125, np.float32), S[:, 1:]], axis=1)
    a = oracle.subcluster_unequal(S, 11)
    b = oracle.subcluster_unequal(Sc, 11)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[3], b[3])
    assert np.all(b[2][:, 1] == np.float32(0.3125))


def test_identical_points_form_one_group(oracle):
    S = np.full((40, 3), 0.75, np.float32)
    perm, offs, _, grp = oracle.subcluster_unequal(S, 5)
    assert np.all(grp == 0)
    np.testing.assert_array_equal(offs, [0, 40, 40, 40, 40, 40])


def test_invalid(oracle):
    S = np.zeros((4, 2), np.float32)
    with pytest.raises(ValueError):
        oracle.subcluster_unequal(S, 0)


# -- the whole method with Algorithm 2 ---------------------------------------

def test_cluster_unequal_structure(oracle):
    X = synth.gaussian_blobs(2000, 4, 6, seed=19)[0]
    N, k_local, m = 250, 20, 9
    r = oracle.cluster(X, N=N, k_local=k_local, k_final=5, max_iter=15, tol=0.0, scheme=1, m=m)
    assert r["T"] == m
    perm, offs, _, grp = oracle.subcluster_unequal(r["S"], m)
    np.testing.assert_array_equal(r["perm"], perm)
    np.testing.assert_array_equal(r["offsets"], offs)
    sizes = np.diff(offs)
    np.testing.assert_array_equal(r["local_k"], -(-sizes * k_local // N))
    assert r["M"] == r["local_k"].sum()
    S = r["S"].astype(np.float64)
    c = 0
    for t in range(m):
        kr = int(r["local_k"][t])
        if kr == 0:
            assert r["local_iters"][t] == 0 and r["local_sse"][t] == 0.0
            continue
        P = S[perm[offs[t]:offs[t + 1]]]
        loc = oracle.lloyd(P, P[:kr], 15, 0.0)
        np.testing.assert_array_equal(loc["centers"], r["local_centers"][c:c + kr])
        assert loc["sse"] == r["local_sse"][t]
        c += kr
    lab, sse, _, _ = oracle.assign(S, r["centers"])
    np.testing.assert_array_equal(lab, r["labels"])
    assert sse == r["sse"]


def test_cluster_unequal_single_group_is_plain_lloyd(oracle):
    X = synth.table1("iris")
    n = len(X)
    r = oracle.cluster(X, N=n, k_local=n, k_final=3, max_iter=40, tol=0.0, scheme=1, m=1)
    S, _, _ = oracle.scale(X)
    stride = n // 3
    direct = oracle.lloyd(S.astype(np.float64), S[::stride][:3], 40, 0.0)
    np.testing.assert_array_equal(r["centers"], direct["centers"])
    np.testing.assert_array_equal(r["labels"], direct["labels"])


def test_cluster_unequal_default_group_count(oracle):
    X = synth.tiny().X[:1000]
    r = oracle.cluster(X, N=300, k_local=32, k_final=5, max_iter=3, tol=0.0, scheme=1)
    assert r["T"] == 4
