"""GPU parity of the unequal sized subclustering (Sec. III, Algorithm 2) and
of the whole method built on it, through the C ABI, against the CPU oracle.

Groups, the permutation, the grouped rows and the binary64 landmarks must
match bit for bit; the local and final Lloyd runs are held to the same
tolerances as with Algorithm 1 (centers and objective 1e-5 relative).
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


def check_unequal(km, oracle, S, m):
    P, perm, offs, lm = km.subcluster_unequal(dev(S), m, landmarks=True)
    permr, offr, lmr, _ = oracle.subcluster_unequal(S, m)
    perm = host(perm)
    assert np.array_equal(host(lm), lmr)
    assert np.array_equal(host(offs), offr)
    assert np.array_equal(perm, permr)
    assert np.array_equal(host(P), S[perm])


@pytest.mark.parametrize("m", [1, 2, 3, 7, 64, 1000, 8192])
def test_unequal_tiny(km, oracle, m):
    S, _, _ = oracle.scale(synth.tiny().X)
    check_unequal(km, oracle, S, m)


@pytest.mark.parametrize("n,d,m", [(1, 1, 1), (1, 3, 5), (2, 1, 2), (10, 3, 4), (4095, 1, 17),
                                   (4097, 4, 33), (9000, 7, 100), (12289, 16, 128),
                                   (3000, 100, 40), (2100, 600, 9), (20000, 2, 2500)])
def test_unequal_shapes(km, oracle, n, d, m):
    # several segments of 4096 points with a ragged tail, float4 and scalar rows
    rng = np.random.default_rng(n + 3 * d + m)
    X = rng.standard_normal((n, d)).astype(np.float32) + rng.integers(0, 4, (n, 1)).astype(np.float32)
    S, _, _ = oracle.scale(X)
    check_unequal(km, oracle, S, m)


def test_unequal_unscaled_input(km, oracle):
    # any finite input: L and H are not 0 and 1
    rng = np.random.default_rng(11)
    S = (rng.standard_normal((7000, 12)) * rng.uniform(0.1, 300, 12) - 40).astype(np.float32)
    for m in (5, 60, 701):
        check_unequal(km, oracle, S, m)


def test_unequal_ties(km, oracle):
    # exact midpoints between landmarks go to the lower landmark
    S = np.array([[0.0], [0.25], [0.75], [1.0], [0.5]], np.float32)
    check_unequal(km, oracle, S, 3)
    # points on the segment, many of them near a midpoint, and duplicates
    rng = np.random.default_rng(5)
    for m in (9, 64, 257):
        t = ((rng.integers(0, m - 1, 6000) + 0.5) / (m - 1)).astype(np.float32)
        S = np.repeat(t[:, None], 8, axis=1)
        S[0], S[1] = 0.0, 1.0
        S[2:200] = S[200:398]
        check_unequal(km, oracle, S, m)


def test_unequal_constant_and_identical(km, oracle):
    rng = np.random.default_rng(6)
    S = rng.uniform(0, 1, (5000, 5)).astype(np.float32)
    S[:, 2] = 0.375
    check_unequal(km, oracle, S, 31)
    check_unequal(km, oracle, np.full((3000, 4), 0.5, np.float32), 12)  # every landmark is L
    # spread far below float32 resolution of the projection in one attribute
    S2 = rng.uniform(0, 1, (4000, 3)).astype(np.float32)
    S2[:, 1] = rng.uniform(0, 1e-30, 4000).astype(np.float32)
    check_unequal(km, oracle, S2, 50)


def test_unequal_mid_workload(km, oracle):
    # 1,048,576 points, d = 16, 1 % outliers, 128 groups
    job = synth.mid()
    S, _, _ = oracle.scale(job.X)
    check_unequal(km, oracle, S, -(-len(S) // job.N))


@pytest.mark.timeout(600)
def test_unequal_precision_workload_sampled(km, oracle):
    # 4,194,304 points, d = 128, 128 groups: landmarks bit-exact from the
    # corner points; the group of sampled points by the oracle's exact
    # assignment against those landmarks; the partition checked everywhere.
    job = synth.precision()
    n, d = job.X.shape
    m = -(-n // job.N)
    S = km.scale(dev(job.X))[0]
    P, perm, offs, lm = km.subcluster_unequal(S, m, landmarks=True)
    Sh, perm, offs, lm = host(S), host(perm), host(offs), host(lm)
    L = Sh.min(axis=0).astype(np.float64)
    H = Sh.max(axis=0).astype(np.float64)
    want = L[None, :] + (np.arange(m, dtype=np.float64) / (m - 1))[:, None] * (H - L)[None, :]
    assert np.array_equal(lm, want)
    assert offs[0] == 0 and offs[-1] == n and np.all(np.diff(offs) >= 0)
    grp = np.repeat(np.arange(m), np.diff(offs))
    assert np.array_equal(np.sort(perm), np.arange(n))
    starts = np.r_[True, np.diff(grp) != 0]
    assert np.all((np.diff(perm) > 0) | starts[1:])  # ascending inside every group
    rng = np.random.default_rng(17)
    pos = rng.choice(n, 4000, replace=False)
    lab, _, _, _ = oracle.assign(Sh[perm[pos]].astype(np.float64), lm)
    assert np.array_equal(lab, grp[pos])
    rows = rng.choice(n, 2000, replace=False)
    assert np.array_equal(host(P)[rows], Sh[perm[rows]])


def test_unequal_rejects_bad_m(km):
    import paper_1412_1947_amd as pkg
    S = dev(np.zeros((10, 2), np.float32))
    for m in (0, 8193):
        with pytest.raises(pkg.SubkmError):
            km.subcluster_unequal(S, m)


# ------------------------------------------------------------- whole method
def check_cluster_unequal(km, oracle, job, m):
    import paper_1412_1947_amd as pkg
    out = km.cluster(dev(job.X), job.N, job.k_local, job.k_final, job.max_iter, job.tol,
                     intermediates=True, stats=True, scheme=pkg.SCHEME_UNEQUAL, m=m)
    ref = oracle.cluster(job.X, job.N, job.k_local, job.k_final, job.max_iter, job.tol,
                         scheme=1, m=m)
    st = out["stats"]
    assert st["T"] == ref["T"] and st["M"] == ref["M"]
    assert np.array_equal(host(out["S"]), ref["S"])
    assert np.array_equal(host(out["perm"]), ref["perm"])
    assert np.array_equal(host(out["local_iters"]), ref["local_iters"])
    assert rel_err(host(out["local_sse"]), ref["local_sse"]) <= TOL
    assert rel_err(host(out["local_centers"])[:ref["M"]], ref["local_centers"]) <= TOL
    assert rel_err(host(out["centers"]), ref["centers"]) <= TOL
    assert abs(host(out["sse"])[0] - ref["sse"]) <= TOL * ref["sse"]
    return out, ref


@pytest.mark.parametrize("m", [0, 3, 9, 40])
def test_cluster_unequal_tiny(km, oracle, m):
    job = synth.tiny()
    out, ref = check_cluster_unequal(km, oracle, job, m)
    assert np.array_equal(host(out["labels"]), ref["labels"])


def test_cluster_unequal_with_empty_groups(km, oracle):
    # two far blobs and many landmarks: most groups stay empty
    rng = np.random.default_rng(21)
    X = np.concatenate([rng.normal(0, 0.05, (1500, 3)), rng.normal(5, 0.05, (1500, 3))]).astype(np.float32)
    job = synth.ClusterJob(X, 300, 30, 4, 15, 0.0)
    out, ref = check_cluster_unequal(km, oracle, job, 64)
    assert np.sum(ref["local_k"] == 0) > 30
    assert np.array_equal(host(out["labels"]), ref["labels"])


def test_cluster_unequal_mid_subset(km, oracle):
    # outliers stretch the segment: unequal groups, one of them large
    job = synth.mid(n=1 << 17)
    job = synth.ClusterJob(job.X, 4096, 128, 32, 10, 1e-6)
    out, ref = check_cluster_unequal(km, oracle, job, 0)
    sizes = np.diff(ref["offsets"])
    assert sizes.max() > 4 * job.N
