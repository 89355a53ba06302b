"""GPU parity of the Manhattan similarity in both subclustering algorithms
(Sec. II names it beside the Euclidean distance), through the C ABI, against
the CPU oracle: subclusters, permutation, grouped rows and landmarks bit for
bit; the whole method to the usual tolerances.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))) if a.size else 0.0


def check_alg1(km, oracle, S, N, mode=0):
    P, perm, offs, lm = km.subcluster(dev(S), N, landmark_mode=mode, landmarks=True, metric=1)
    permr, offr, lmr = oracle.subcluster(S, N, fixed_landmark=bool(mode), metric=1)
    perm = host(perm)
    assert np.array_equal(host(offs), offr)
    assert np.array_equal(host(lm), lmr)
    assert np.array_equal(perm, permr)
    assert np.array_equal(host(P), S[perm])


def check_alg2(km, oracle, S, m):
    P, perm, offs, lm = km.subcluster_unequal(dev(S), m, landmarks=True, metric=1)
    permr, offr, lmr, _ = oracle.subcluster_unequal(S, m, metric=1)
    perm = host(perm)
    assert np.array_equal(host(lm), lmr)
    assert np.array_equal(host(offs), offr)
    assert np.array_equal(perm, permr)
    assert np.array_equal(host(P), S[perm])


@pytest.mark.parametrize("N", [1, 100, 512, 4096])
def test_alg1_tiny(km, oracle, N):
    S, _, _ = oracle.scale(synth.tiny().X)
    check_alg1(km, oracle, S, N)


@pytest.mark.parametrize("n,d,N", [(10, 3, 4), (3000, 1, 200), (6000, 3, 777), (5000, 16, 2048),
                                   (2100, 600, 700)])
def test_alg1_shapes(km, oracle, n, d, N):
    rng = np.random.default_rng(n + d + N + 5)
    X = rng.standard_normal((n, d)).astype(np.float32) + rng.integers(0, 4, (n, 1)).astype(np.float32)
    S, _, _ = oracle.scale(X)
    check_alg1(km, oracle, S, N)


@pytest.mark.parametrize("mode", [0, 1])
def test_alg1_ties(km, oracle, mode):
    rng = np.random.default_rng(4)
    S = (rng.integers(0, 3, (9000, 2)) / 2).astype(np.float32)
    check_alg1(km, oracle, S, 1000, mode)


def test_alg1_mid_subset(km, oracle):
    job = synth.mid(n=1 << 18)
    S, _, _ = oracle.scale(job.X)
    check_alg1(km, oracle, S, job.N)


@pytest.mark.parametrize("m", [1, 3, 64, 1000])
def test_alg2_tiny(km, oracle, m):
    S, _, _ = oracle.scale(synth.tiny().X)
    check_alg2(km, oracle, S, m)


@pytest.mark.parametrize("n,d,m", [(4097, 4, 33), (9000, 7, 100), (3000, 100, 40), (2100, 600, 9)])
def test_alg2_shapes(km, oracle, n, d, m):
    rng = np.random.default_rng(n + 3 * d + m + 1)
    X = rng.standard_normal((n, d)).astype(np.float32) + rng.integers(0, 4, (n, 1)).astype(np.float32)
    S, _, _ = oracle.scale(X)
    check_alg2(km, oracle, S, m)


def test_alg2_unscaled_and_mid(km, oracle):
    rng = np.random.default_rng(12)
    S = (rng.standard_normal((7000, 12)) * rng.uniform(0.1, 300, 12) - 40).astype(np.float32)
    check_alg2(km, oracle, S, 60)
    job = synth.mid(n=1 << 18)
    S2, _, _ = oracle.scale(job.X)
    check_alg2(km, oracle, S2, 32)


def test_measure_switch_on_same_buffers(km, oracle):
    # the captured subclustering sequence is cached per configuration: the
    # measure must select its own sequence
    S, _, _ = oracle.scale(synth.tiny().X)
    Sd = dev(S)
    for metric in (0, 1, 0, 1):
        _, perm, _ = km.subcluster(Sd, 300, metric=metric)
        assert np.array_equal(host(perm), oracle.subcluster(S, 300, metric=metric)[0])


@pytest.mark.parametrize("scheme", [0, 1])
def test_cluster_manhattan(km, oracle, scheme):
    job = synth.tiny()
    out = km.cluster(dev(job.X), job.N, job.k_local, job.k_final, job.max_iter, job.tol,
                     intermediates=True, stats=True, scheme=scheme, metric=1)
    ref = oracle.cluster(job.X, job.N, job.k_local, job.k_final, job.max_iter, job.tol,
                         scheme=scheme, metric=1)
    assert out["stats"]["T"] == ref["T"] and out["stats"]["M"] == ref["M"]
    assert np.array_equal(host(out["perm"]), ref["perm"])
    assert rel_err(host(out["local_centers"])[:ref["M"]], ref["local_centers"]) <= TOL
    assert rel_err(host(out["centers"]), ref["centers"]) <= TOL
    assert np.array_equal(host(out["labels"]), ref["labels"])
    assert abs(host(out["sse"])[0] - ref["sse"]) <= TOL * ref["sse"]


def test_rejects_unknown_metric(km):
    import paper_1412_1947_amd as pkg
    S = dev(np.zeros((10, 2), np.float32))
    with pytest.raises(pkg.SubkmError):
        km.subcluster(S, 5, metric=2)
    with pytest.raises(pkg.SubkmError):
        km.subcluster_unequal(S, 5, metric=-1)
