"""Pins of the oracle's whole two-level method (Sec. II Algorithm 1 with the
final clustering of the local centers described in Sec. I and Sec. V).

With one subcluster holding every point and as many local centers as points,
the local stage is the identity, so the method must reduce to plain Lloyd on
the scaled points from the strided start; the structural facts (subcluster
sizes, local center counts, the compression value N / k_local) are checked on
shape stand-ins of the paper's workloads.
"""
import numpy as np
import pytest

import synth


def test_reduces_to_plain_lloyd(oracle):
    X = synth.table1("seeds")
    n = len(X)
    r = oracle.cluster(X, N=n, k_local=n, k_final=3, max_iter=40, tol=0.0)
    S, _, _ = oracle.scale(X)
    assert r["T"] == 1 and r["M"] == n
    np.testing.assert_array_equal(r["local_centers"], S.astype(np.float64))
    stride = n // 3
    direct = oracle.lloyd(S.astype(np.float64), S[::stride][:3], 40, 0.0)
    np.testing.assert_array_equal(r["centers"], direct["centers"])
    np.testing.assert_array_equal(r["labels"], direct["labels"])
    assert r["sse"] == direct["sse"]


@pytest.mark.parametrize("which,N,k_local", [("iris", 25, 5), ("seeds", 35, 6)])
def test_structure_table1_shapes(oracle, which, N, k_local):
    X = synth.table1(which)
    n = len(X)
    r = oracle.cluster(X, N=N, k_local=k_local, k_final=3, max_iter=20, tol=0.0)
    assert r["T"] == 6
    np.testing.assert_array_equal(np.diff(r["offsets"]), N)
    np.testing.assert_array_equal(r["local_k"], k_local)
    assert r["M"] == 6 * k_local
    assert np.all(np.bincount(r["labels"], minlength=3) > 0)
    # each local run is an ordinary Lloyd run on its subcluster from its first points
    S = r["S"].astype(np.float64)
    for t in range(r["T"]):
        P = S[r["perm"][r["offsets"][t]:r["offsets"][t + 1]]]
        loc = oracle.lloyd(P, P[:k_local], 20, 0.0)
        np.testing.assert_array_equal(loc["centers"], r["local_centers"][t * k_local:(t + 1) * k_local])
        assert loc["sse"] == r["local_sse"][t]
    # labels and objective are those of the final centers
    lab, sse, _, _ = oracle.assign(S, r["centers"])
    np.testing.assert_array_equal(lab, r["labels"])
    assert sse == r["sse"]


def test_partial_last_subcluster(oracle):
    X = synth.tiny().X[:1000]
    r = oracle.cluster(X, N=300, k_local=32, k_final=5, max_iter=5, tol=0.0)
    assert r["T"] == 4
    np.testing.assert_array_equal(np.diff(r["offsets"]), [300, 300, 300, 100])
    np.testing.assert_array_equal(r["local_k"], [32, 32, 32, 11])  # ceil(100*32/300)
    assert r["M"] == 107


def test_tiny_workload_runs(oracle):
    job = synth.tiny()
    r = oracle.cluster(job.X, job.N, job.k_local, job.k_final, job.max_iter, job.tol)
    assert r["T"] == 8 and r["M"] == 256
    np.testing.assert_array_equal(r["local_iters"], 20)
    assert r["final_iters"] == 20
    # two-level clustering of 8 well-separated blobs: every blob lands in one cluster
    assert r["sse"] > 0


def test_invalid(oracle):
    X = synth.tiny().X[:100]
    with pytest.raises(ValueError):
        oracle.cluster(X, N=10, k_local=11, k_final=2, max_iter=1, tol=0)  # k_local > N
    with pytest.raises(ValueError):
        oracle.cluster(X, N=100, k_local=2, k_final=3, max_iter=1, tol=0)  # k_final > M
