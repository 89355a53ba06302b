"""Degenerate and boundary cases of the whole method against the oracle:
one point, one subcluster, every point its own local center, as many final
centers as local ones, no moves at all, the widest rows, identical points,
more groups than points, and inputs the calls must refuse.
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


def check(km, oracle, X, N, kl, kf, it, tol, scheme=0, m=0):
    out = km.cluster(dev(X), N, kl, kf, it, tol, intermediates=True, stats=True, scheme=scheme, m=m)
    ref = oracle.cluster(X, N, kl, kf, it, tol, scheme=scheme, m=m)
    st = out["stats"]
    assert st["T"] == ref["T"] and st["M"] == ref["M"]
    assert np.array_equal(host(out["S"]), ref["S"])
    assert np.array_equal(host(out["perm"]), ref["perm"])
    assert np.array_equal(host(out["local_iters"]), ref["local_iters"])
    assert rel_err(host(out["local_centers"])[:ref["M"]], ref["local_centers"]) <= TOL
    assert rel_err(host(out["centers"]), ref["centers"]) <= TOL
    assert np.array_equal(host(out["labels"]), ref["labels"])
    assert abs(host(out["sse"])[0] - ref["sse"]) <= TOL * max(ref["sse"], 1e-30)
    return out, ref


def test_single_point(km, oracle):
    X = np.array([[1.5, -2.0, 7.0]], np.float32)
    out, ref = check(km, oracle, X, 1, 1, 1, 10, 0.0)
    assert ref["sse"] == 0.0


def test_one_subcluster(km, oracle):
    X = synth.tiny().X[:3000]
    check(km, oracle, X, 10_000, 100, 7, 15, 0.0)  # N > n: T = 1, k_r = 30


def test_every_point_its_own_center(km, oracle):
    X = synth.tiny().X[:1200]
    out, ref = check(km, oracle, X, 300, 300, 5, 10, 0.0)  # k_local = N: local stage is the identity
    assert ref["M"] == 1200
    assert np.all(ref["local_sse"] == 0.0)


def test_as_many_final_centers_as_local(km, oracle):
    X = synth.tiny().X[:2000]
    M = 5 * 40  # T = 5 subclusters of 400 points, 40 centers each
    out, ref = check(km, oracle, X, 400, 40, M, 10, 0.0)
    assert ref["M"] == M


def test_no_moves(km, oracle):
    X = synth.tiny().X[:2500]
    out, ref = check(km, oracle, X, 512, 32, 8, 0, 0.0)
    assert np.all(ref["local_iters"] == 0) and ref["final_iters"] == 0


def test_widest_rows(km, oracle):
    rng = np.random.default_rng(4096)
    X = (rng.standard_normal((260, 4096)) + rng.integers(0, 3, (260, 1))).astype(np.float32)
    check(km, oracle, X, 100, 10, 3, 5, 0.0)


def test_identical_points(km, oracle):
    X = np.full((3000, 6), 2.5, np.float32)
    out, ref = check(km, oracle, X, 700, 20, 4, 10, 0.0)
    assert ref["sse"] == 0.0


def test_more_groups_than_points(km, oracle):
    X = synth.tiny().X[:50]
    check(km, oracle, X, 10, 2, 3, 10, 0.0, scheme=1, m=200)


def test_refused_inputs(km):
    import paper_1412_1947_amd as pkg
    X = dev(np.zeros((0, 3), np.float32))
    with pytest.raises(pkg.SubkmError):
        km.cluster(X, 10, 2, 2, 5, 0.0)
    Y = dev(np.ones((100, 3), np.float32))
    with pytest.raises(pkg.SubkmError):
        km.cluster(Y, 10, 11, 2, 5, 0.0)  # k_local > N
    with pytest.raises(pkg.SubkmError):
        km.cluster(Y, 10, 2, 21, 5, 0.0)  # k_final > M = 20
    with pytest.raises(pkg.SubkmError):
        km.cluster(Y, 10, 2, 2, -1, 0.0)  # negative max_iter
    with pytest.raises(pkg.SubkmError):
        km.cluster(Y, 10, 2, 2, 5, float("nan"))
    bad = np.ones((100, 3), np.float32)
    bad[7, 1] = np.nan
    with pytest.raises(pkg.SubkmError):
        km.cluster(dev(bad), 10, 2, 2, 5, 0.0)
