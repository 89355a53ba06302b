"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Scaling and subclustering must match bit for bit.  Lloyd is checked step by
step ("shadow" parity: the oracle takes the GPU's float32 centers as its
input), where labels must match exactly -- the library re-assigns every
point whose two nearest centers are within its float32 error bound with
binary64 distances -- and centers and objective within 1e-5 relative.
"""
import numpy as np
import pytest
import torch

import protocol
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


# ----------------------------------------------------------------------------- scale
@pytest.mark.parametrize("n,d", [(1, 1), (7, 3), (4096, 4), (5000, 7), (3001, 64), (1000, 100),
                                 (257, 300), (500, 65), (700, 130), (9, 1030), (40000, 128)])
def test_scale_bit_exact(km, oracle, n, d):
    rng = np.random.default_rng(n * 31 + d)
    X = (rng.standard_normal((n, d)) * rng.uniform(0.01, 100, d) + rng.uniform(-9, 9, d)).astype(np.float32)
    if d > 2:
        X[:, 1] = 0.625  # constant attribute
    S, mn, mx = km.scale(dev(X))
    Sr, mnr, mxr = oracle.scale(X)
    assert np.array_equal(host(mn), mnr) and np.array_equal(host(mx), mxr)
    assert np.array_equal(host(S), Sr)


def test_scale_mid_workload(km, oracle):
    X = synth.mid(n=1 << 18).X
    S, _, _ = km.scale(dev(X))
    assert np.array_equal(host(S), oracle.scale(X)[0])


def test_scale_rejects_nan(km):
    import paper_1412_1947_amd as pkg
    X = np.ones((100, 4), np.float32)
    X[50, 2] = np.nan
    with pytest.raises(pkg.SubkmError) as e:
        km.scale(dev(X))
    assert e.value.status == 1


# ------------------------------------------------------------------------ subcluster
def check_subcluster(km, oracle, S, N, mode=0):
    P, perm, offs, lm = km.subcluster(dev(S), N, landmark_mode=mode, landmarks=True)
    permr, offr, lmr = oracle.subcluster(S, N, fixed_landmark=bool(mode))
    perm = host(perm)
    assert np.array_equal(host(offs), offr)
    assert np.array_equal(host(lm), lmr)
    assert np.array_equal(perm, permr)
    assert np.array_equal(host(P), S[perm])


@pytest.mark.parametrize("N", [1, 7, 100, 512, 1000, 4095, 4096, 10 ** 6])
def test_subcluster_tiny(km, oracle, N):
    S, _, _ = oracle.scale(synth.tiny().X)
    check_subcluster(km, oracle, S, N)


@pytest.mark.parametrize("n,d,N", [(1, 1, 1), (2, 1, 1), (10, 3, 4), (3000, 1, 200), (6000, 3, 777),
                                   (5000, 16, 2048), (4000, 100, 999), (2100, 600, 700),
                                   (20000, 2, 2500)])
def test_subcluster_shapes(km, oracle, n, d, N):
    rng = np.random.default_rng(n + d + N)
    X = rng.standard_normal((n, d)).astype(np.float32) + rng.integers(0, 4, (n, 1)).astype(np.float32)
    S, _, _ = oracle.scale(X)
    check_subcluster(km, oracle, S, N)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 8, 12, 16, 32, 33, 64, 128])
@pytest.mark.parametrize("aligned", [True, False])
def test_subcluster_row_widths(km, oracle, d, aligned):
    # the keys pass and the compaction have specialised forms per row width
    # and alignment (float4 rows for d = 4, 8, 16, 32 on 16-byte boundaries,
    # single words for d = 1, 2, 4, 8 otherwise) and general ones (the other
    # widths, 64 and 128 among them); several blocks of 2048 positions, a
    # ragged last block, the last round taking everything
    n, N = 9001, 1100
    rng = np.random.default_rng(70 + d)
    X = rng.standard_normal((n, d)).astype(np.float32) + rng.integers(0, 4, (n, 1)).astype(np.float32)
    S, _, _ = oracle.scale(X)
    buf = torch.zeros(n * d + 1, dtype=torch.float32, device="cuda:0")
    Sd = buf[(0 if aligned else 1):][:n * d].view(n, d)
    Sd.copy_(dev(S))
    assert (Sd.data_ptr() % 16 == 0) == aligned
    for mode in (0, 1):
        P, perm, offs, lm = km.subcluster(Sd, N, landmark_mode=mode, landmarks=True)
        permr, offr, lmr = oracle.subcluster(S, N, fixed_landmark=bool(mode))
        perm = host(perm)
        assert np.array_equal(host(offs), offr)
        assert np.array_equal(host(lm), lmr)
        assert np.array_equal(perm, permr)
        assert np.array_equal(host(P), S[perm])


def test_subcluster_graph_cache(km, oracle):
    # the captured subclustering sequences are cached per configuration (8
    # at most, least recently used replaced): ten configurations on the same
    # buffers, cycled twice, hit and evict entries; every result must be the
    # oracle's
    S, _, _ = oracle.scale(synth.tiny().X)
    Sd = dev(S)
    Ns = [100, 150, 200, 300, 450, 512, 700, 1000, 1500, 2048]
    refs = {N: oracle.subcluster(S, N) for N in Ns}
    for rep in range(2):
        for N in Ns + Ns[::-1][:3]:
            P, perm, offs = km.subcluster(Sd, N)
            permr, offr, _ = refs[N]
            assert np.array_equal(host(perm), permr)
            assert np.array_equal(host(offs), offr)
            assert np.array_equal(host(P), S[permr])


@pytest.mark.parametrize("mode", [0, 1])
def test_subcluster_threshold_jumps(km, oracle, mode):
    # the selection histogram of a round is centred on the previous round's
    # threshold; thresholds that jump by many binades from one round to the
    # next (up: a tight cluster at the corner, then a wide cloud; down: a
    # sparse cloud, then near-duplicates) land in its clamped end bins, where
    # the exact path must still hold
    rng = np.random.default_rng(44)
    tight = rng.normal(0.0, 1e-5, (3000, 3))
    wide = rng.uniform(0.5, 3.0, (4000, 3))
    S = np.concatenate([wide[:2000], tight, wide[2000:]]).astype(np.float32)
    check_subcluster(km, oracle, S, 1000, mode)
    sparse = rng.uniform(0.0, 1.0, (2500, 4))
    dup = np.repeat(rng.uniform(0.9, 0.9001, (30, 4)), 100, axis=0) + rng.normal(0, 1e-7, (3000, 4))
    S2 = np.concatenate([dup[:1500], sparse, dup[1500:]]).astype(np.float32)
    check_subcluster(km, oracle, S2, 700, mode)


@pytest.mark.parametrize("mode", [0, 1])
def test_subcluster_ties_and_duplicates(km, oracle, mode):
    rng = np.random.default_rng(3)
    S = (rng.integers(0, 3, (9000, 2)) / 2).astype(np.float32)  # 9 distinct points only
    check_subcluster(km, oracle, S, 1000, mode)
    S2 = np.repeat(rng.uniform(0, 1, (40, 4)).astype(np.float32), 100, axis=0)
    check_subcluster(km, oracle, S2, 333, mode)


def test_subcluster_fixed_landmark(km, oracle):
    S, _, _ = oracle.scale(synth.tiny().X)
    check_subcluster(km, oracle, S, 300, mode=1)


def test_subcluster_mid_workload(km, oracle):
    job = synth.mid(n=1 << 18)
    S, _, _ = oracle.scale(job.X)
    check_subcluster(km, oracle, S, job.N)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,d,metric", [(600_001, 2, 0), (300_000, 8, 0), (600_000, 32, 0),
                                        (300_001, 1, 0), (600_000, 16, 1), (530_000, 4, 1)])
def test_subcluster_many_points_per_thread(km, oracle, n, d, metric):
    # above 2^18 and 2^19 remaining points the keys pass gives each thread 2
    # or 4 points; every row width of that form, both measures
    X, _ = synth.gaussian_blobs(n, d, 20, seed=n + d, sigma=0.4)
    S, _, _ = oracle.scale(X)
    N = 8192
    P, perm, offs, lm = km.subcluster(dev(S), N, landmarks=True, metric=metric)
    permr, offr, lmr = oracle.subcluster(S, N, metric=metric)
    assert np.array_equal(host(lm), lmr)
    assert np.array_equal(host(perm), permr)
    assert np.array_equal(host(P), S[permr])


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,d,metric,mode", [(300_000, 16, 0, 0), (200_000, 8, 1, 0),
                                             (250_000, 16, 0, 1), (150_000, 64, 0, 0),
                                             (70_000, 128, 1, 0), (90_000, 100, 0, 0)])
def test_subcluster_tied_minimum_holders(km, oracle, n, d, metric, mode):
    # values on a 1/8 grid (many keys tie), and below it, per attribute, five
    # levels held by two random points each: rounds where some holder of
    # the current minimum stays (the compaction reads only the selected
    # rows) alternate with rounds where the last ones leave and the landmark
    # moves (a third of the rounds here); with a fixed landmark no row that
    # stays is read at all.  Rows of 64 to 128 attributes take the staged
    # keys pass, which folds the rows above the previous round's bound into
    # the next landmark (several tiles per block at these sizes)
    rng = np.random.default_rng(n + d + mode)
    X = (np.floor(rng.beta(2.0, 5.0, (n, d)) * 8.0) / 8.0).astype(np.float32)
    for j in range(d):
        for level in range(1, 6):
            X[rng.integers(0, n, 2), j] = -level / 8.0
    S, _, _ = oracle.scale(X)
    N = 4096
    P, perm, offs, lm = km.subcluster(dev(S), N, landmark_mode=mode, landmarks=True, metric=metric)
    permr, offr, lmr = oracle.subcluster(S, N, fixed_landmark=bool(mode), metric=metric)
    assert np.array_equal(host(lm), lmr)
    assert np.array_equal(host(perm), permr)
    assert np.array_equal(host(P), S[permr])


@pytest.mark.parametrize("mode", [0, 1])
def test_subcluster_batched_rounds(km, oracle, mode):
    # consecutive rounds that share a landmark are selected in one pass (at
    # most 9 rounds, the last round on its own): with a fixed landmark every
    # pass but the last takes 9; with the attribute-wise minimum, rounds
    # join while some point holding each attribute's minimum surely stays.
    # The subclusters stay those of the oracle, bit for bit.
    job = synth.mid(n=1 << 17)
    N = 1024
    out = km.cluster(dev(job.X), N=N, k_local=8, k_final=4, max_iter=1, tol=0.0, landmark_mode=mode,
                     intermediates=True, stats=True)
    T = out["stats"]["T"]
    S, _, _ = oracle.scale(job.X)
    assert np.array_equal(host(out["S"]), S)
    permr, _, _ = oracle.subcluster(S, N, fixed_landmark=bool(mode))
    assert np.array_equal(host(out["perm"]), permr)
    nsel = out["stats"]["sub_selections"]
    if mode == 1:
        assert nsel == -(-(T - 1) // 9)
    else:
        assert -(-(T - 1) // 9) <= nsel < T - 1


# ----------------------------------------------------------------------------- Lloyd
def shadow_steps(km, oracle, X, C0, steps, precision=0):
    """Run `steps` single GPU iterations, each checked against one oracle
    iteration from the same float32 centers."""
    n, d = X.shape
    k = C0.shape[0]
    Xd = dev(X)
    X64 = X.astype(np.float64)
    C = C0.astype(np.float32).copy()
    lab_d = torch.empty(n, dtype=torch.int32, device="cuda:0")
    # max_iter = 0: a pure assignment
    Cd = dev(C)
    _, sse = km.lloyd_batched(Xd, [(0, n, 0, 0, d, k)], Cd, lab_d, 0, 0.0, precision)
    lab_r, sse_r, _, _ = oracle.assign(X64, C)
    assert np.array_equal(host(lab_d), lab_r)
    assert abs(host(sse)[0] - sse_r) <= TOL * sse_r + 1e-300
    for _ in range(steps):
        Cd = dev(C)
        it, sse = km.lloyd_batched(Xd, [(0, n, 0, 0, d, k)], Cd, lab_d, 1, 0.0, precision)
        Cg = host(Cd)
        lab0, _, _, _ = oracle.assign(X64, C)
        Cref, _, _ = oracle.update(X64, lab0, C.astype(np.float64))
        assert rel_err(Cg, Cref) <= TOL
        lab1, sse1, _, _ = oracle.assign(X64, Cg)
        assert np.array_equal(host(lab_d), lab1)
        assert abs(host(sse)[0] - sse1) <= TOL * sse1
        assert host(it)[0] == 1
        C = Cg


@pytest.mark.parametrize("n,d,k", [(512, 4, 32), (1000, 2, 10), (3000, 16, 256), (2000, 7, 50),
                                   (777, 32, 77), (1500, 64, 100), (900, 128, 300), (300, 3, 300)])
def test_lloyd_shadow(km, oracle, n, d, k):
    rng = np.random.default_rng(n * 7 + d)
    X, _ = synth.gaussian_blobs(n, d, max(2, k // 8), seed=n + d, sigma=0.7)
    S, _, _ = oracle.scale(X)
    shadow_steps(km, oracle, S, S[:k], steps=3)


def test_lloyd_ties_and_empty_clusters(km, oracle):
    # duplicated points and duplicated centers: exact ties everywhere; the
    # second copy of every center ends up empty and must stay in place
    rng = np.random.default_rng(11)
    base = rng.uniform(0, 1, (20, 3)).astype(np.float32)
    X = np.repeat(base, 30, axis=0)
    C0 = np.concatenate([base[:10], base[:10]])
    shadow_steps(km, oracle, X, C0, steps=2)


def test_lloyd_k1_and_k_equals_n(km, oracle):
    X, _ = synth.gaussian_blobs(200, 5, 3, seed=5)
    S, _, _ = oracle.scale(X)
    shadow_steps(km, oracle, S, S[:1], steps=1)
    shadow_steps(km, oracle, S[:50], S[:50], steps=1)


def run_batch(km, runs_np, ks, max_iter, tol, form=0, precision=0, pad=0):
    """Many runs in one call (the points start `pad` floats into the buffer);
    returns per-run centers, labels, iters, sse."""
    xs, specs, x_off, c_off, l_off = [np.zeros(pad, np.float32)], [], pad, 0, 0
    for X, k in zip(runs_np, ks):
        n, d = X.shape
        specs.append((x_off, n, c_off, l_off, d, k))
        xs.append(X.reshape(-1))
        x_off += n * d
        c_off += k * d
        l_off += n
    P = dev(np.concatenate(xs))
    C = torch.cat([dev(X[:k].reshape(-1)) for X, k in zip(runs_np, ks)])
    lab = torch.empty(l_off, dtype=torch.int32, device="cuda:0")
    it, sse = km.lloyd_batched(P, specs, C, lab, max_iter, tol, precision, form)
    Ch, labh, ith, sseh = host(C), host(lab), host(it), host(sse)
    out = []
    for (xo, n, co, lo, d, k) in specs:
        out.append((Ch[co:co + k * d].reshape(k, d), labh[lo:lo + n]))
    return out, ith, sseh


def test_lloyd_batched_matches_oracle_trajectory(km, oracle):
    # whole runs against the oracle's own trajectories (the comparison
    # protocol of tests/protocol.py): every run free of near ties must give
    # the oracle's centers, objective and move count; at least 10 of the 12
    # runs are such runs here; every run passes the shadow step
    rng = np.random.default_rng(21)
    runs, ks = [], []
    for j in range(12):
        n = int(rng.integers(300, 3000))
        d = int(rng.choice([2, 4, 8, 16, 5]))
        X, _ = synth.gaussian_blobs(n, d, int(rng.integers(3, 12)), seed=j, sigma=0.4)
        runs.append(oracle.scale(X)[0])
        ks.append(int(rng.integers(1, 40)))
    out, iters, sse = run_batch(km, runs, ks, 15, 1e-6)
    trajs = protocol.trajectories(oracle, [(X.astype(np.float64), X[:k]) for X, k in zip(runs, ks)],
                                  15, 1e-6)
    compared = 0
    for r, (X, k) in enumerate(zip(runs, ks)):
        C, lab = out[r]
        ref = oracle.lloyd(X.astype(np.float64), X[:k], 15, 1e-6)
        # the step-by-step trajectory is oracle.lloyd itself
        assert np.array_equal(ref["centers"], trajs[r]["centers"]) and ref["iters"] == trajs[r]["iters"]
        if protocol.check_independent(C, sse[r], iters[r], trajs[r], 1e-6, f"run {r}"):
            compared += 1
            if iters[r] == trajs[r]["iters"]:
                assert np.array_equal(lab, trajs[r]["labels"]), r
    assert compared >= 10, compared
    protocol.shadow(km, oracle, runs, [o[0] for o in out], what="trajectory runs")


def test_back_to_back_calls_without_sync(km, oracle):
    # the calls never synchronise: a long call first (its work keeps the
    # stream busy, so the plan copies of the calls after it queue behind
    # it), then eight batched calls with different run layouts issued back
    # to back, more than the four slots of the plan staging ring; each must
    # give the bits of the same call made alone, with a sync after it
    rng = np.random.default_rng(9)
    cases = []
    for j in range(8):
        runs, ks = [], []
        for q in range(int(rng.integers(1, 6))):
            n = int(rng.integers(200, 4000))
            d = int(rng.choice([4, 8, 16, 32]))
            X, _ = synth.gaussian_blobs(n, d, 6, seed=900 + 10 * j + q, sigma=0.5)
            runs.append(oracle.scale(X)[0])
            ks.append(int(rng.integers(2, min(n, 200))))
        cases.append((runs, ks))

    def prepare(runs, ks):
        # device buffers made up front: torch's copies from host memory
        # synchronise, the library's calls must not
        specs, x_off, c_off, l_off = [], 0, 0, 0
        for X, k in zip(runs, ks):
            n, d = X.shape
            specs.append((x_off, n, c_off, l_off, d, k))
            x_off, c_off, l_off = x_off + n * d, c_off + k * d, l_off + n
        P = torch.cat([dev(X.reshape(-1)) for X in runs])
        C0 = torch.cat([dev(X[:k].reshape(-1)) for X, k in zip(runs, ks)])
        return specs, P, C0, l_off

    def issue(specs, P, C0, l_off):
        C = C0.clone()
        lab = torch.empty(l_off, dtype=torch.int32, device="cuda:0")
        it, sse = km.lloyd_batched(P, specs, C, lab, 12, 1e-6)
        return C, lab, it, sse

    bufs = [prepare(runs, ks) for runs, ks in cases]
    alone = []
    for b in bufs:
        r = issue(*b)
        torch.cuda.synchronize()
        alone.append([host(t) for t in r])
    big = synth.mid(n=1 << 18)
    Sb = oracle.scale(big.X)[0]
    nb = Sb.shape[0] // 32
    long_specs = [(q * nb * 16, nb, q * 256 * 16, q * nb, 16, 256) for q in range(32)]
    Cl = torch.cat([dev(Sb[q * nb:q * nb + 256].reshape(-1)) for q in range(32)])
    lab_l = torch.empty(Sb.shape[0], dtype=torch.int32, device="cuda:0")
    Pl = dev(Sb.reshape(-1))
    torch.cuda.synchronize()
    km.lloyd_batched(Pl, long_specs, Cl, lab_l, 30, 0.0)
    queued = [issue(*b) for b in bufs]
    torch.cuda.synchronize()
    km.synchronize()
    for j, (q, a) in enumerate(zip(queued, alone)):
        for t, ref in zip(q, a):
            assert np.array_equal(host(t), ref), j


def test_plain_equals_batched_and_deterministic(km, oracle):
    rng = np.random.default_rng(5)
    runs, ks = [], []
    for j in range(9):
        n = int(rng.integers(100, 5000))
        X, _ = synth.gaussian_blobs(n, 16, 10, seed=100 + j, sigma=0.5)
        runs.append(oracle.scale(X)[0])
        ks.append(int(min(n, rng.integers(1, 300))))
    a, ia, sa = run_batch(km, runs, ks, 10, 1e-6, form=0)
    b, ib, sb = run_batch(km, runs, ks, 10, 1e-6, form=1)
    c, ic, sc = run_batch(km, runs, ks, 10, 1e-6, form=0)
    assert np.array_equal(ia, ib) and np.array_equal(sa, sb) and np.array_equal(sa, sc)
    for (ca, la), (cb, lb), (cc, lc) in zip(a, b, c):
        assert np.array_equal(ca, cb) and np.array_equal(la, lb)
        assert np.array_equal(ca, cc) and np.array_equal(la, lc)


@pytest.mark.parametrize("n,k,d", [(32768, 64, 16), (12000, 64, 16), (20000, 100, 8),
                                   (30001, 16, 4), (9000, 64, 32)])
def test_forms_agree_on_long_runs(km, oracle, n, k, d):
    # runs long enough to be split over many blocks of the persistent kernel
    # (they reduce-scatter their partial sums, in slices that need not
    # divide the sums evenly); the plain form sums through global integer
    # atomics instead, so equal bits show the exchange is exact; the batched
    # result alone and next to short runs in the same call
    X, _ = synth.gaussian_blobs(n, d, 2 * k, seed=n + k, sigma=0.4)
    S = oracle.scale(X)[0]
    a, ia, sa = run_batch(km, [S], [k], 8, 0.0, form=0)
    b, ib, sb = run_batch(km, [S], [k], 8, 0.0, form=1)
    assert np.array_equal(ia, ib) and np.array_equal(sa, sb)
    assert np.array_equal(a[0][0], b[0][0]) and np.array_equal(a[0][1], b[0][1])
    short = [oracle.scale(synth.gaussian_blobs(700, d, 5, seed=j, sigma=0.5)[0])[0] for j in range(3)]
    c, ic, sc = run_batch(km, short + [S], [20, 20, 20, k], 8, 0.0, form=0)
    assert np.array_equal(c[3][0], a[0][0]) and np.array_equal(c[3][1], a[0][1]) and sc[3] == sa[0]
    # moves one at a time against the oracle (each goes through the exchange)
    shadow_steps(km, oracle, S, S[:k], steps=2)


# --------------------------------------------------------------------------- cluster
def check_cluster(km, oracle, job, fixed=False):
    X = dev(job.X)
    out = km.cluster(X, job.N, job.k_local, job.k_final, job.max_iter, job.tol,
                     landmark_mode=int(fixed), intermediates=True, stats=True)
    ref = oracle.cluster(job.X, job.N, job.k_local, job.k_final, job.max_iter, job.tol,
                         fixed_landmark=fixed)
    assert np.array_equal(host(out["S"]), ref["S"])
    assert np.array_equal(host(out["perm"]), ref["perm"])
    st = out["stats"]
    assert st["T"] == ref["T"] and st["M"] == ref["M"]
    loc = host(out["local_centers"])
    return out, ref, loc


def test_cluster_tiny_end_to_end(km, oracle):
    job = synth.tiny()
    out, ref, loc = check_cluster(km, oracle, job)
    assert rel_err(loc, ref["local_centers"]) <= TOL
    assert np.array_equal(host(out["local_iters"]), ref["local_iters"])
    assert rel_err(host(out["local_sse"]), ref["local_sse"]) <= TOL
    assert rel_err(host(out["centers"]), ref["centers"]) <= TOL
    assert np.array_equal(host(out["labels"]), ref["labels"])
    assert abs(host(out["sse"])[0] - ref["sse"]) <= TOL * ref["sse"]


@pytest.mark.parametrize("which,N,k_local", [("iris", 25, 5), ("seeds", 35, 6)])
def test_cluster_table1_shapes(km, oracle, which, N, k_local):
    job = synth.ClusterJob(synth.table1(which), N, k_local, 3, 20, 0.0)
    out, ref, loc = check_cluster(km, oracle, job)
    assert rel_err(loc, ref["local_centers"]) <= TOL
    assert abs(host(out["sse"])[0] - ref["sse"]) <= TOL * ref["sse"]


def test_cluster_ragged_tail_and_fixed_landmark(km, oracle):
    X = synth.tiny().X[:3333]
    job = synth.ClusterJob(X, 500, 20, 6, 12, 0.0)
    check_cluster(km, oracle, job, fixed=True)
    out, ref, loc = check_cluster(km, oracle, job)
    assert rel_err(loc, ref["local_centers"]) <= TOL


# ------------------------------------------------------- chunked path, ragged runs
def test_ragged_large_k_runs(km, oracle):
    """Runs whose k*d exceeds the LDS budget (centers streamed in chunks,
    label-scan update), mixed with small runs and two attribute counts in one
    call; every run is checked step by step against the oracle."""
    rng = np.random.default_rng(33)
    runs, ks = [], []
    for j, (n, d) in enumerate([(6000, 32), (3000, 8), (9000, 32), (1500, 8), (2500, 32), (700, 5)]):
        X, _ = synth.gaussian_blobs(n, d, int(rng.integers(4, 33)), seed=300 + j, sigma=(0.2, 1.5))
        runs.append(oracle.scale(X)[0])
        ks.append(int(min(-(-n // 32) * 4, 1024)) if d == 32 else int(-(-n // 32)))
    # one batched call, 3 moves, then one more move checked against the oracle
    out, iters, sse = run_batch(km, runs, ks, 3, 0.0)
    for r, (X, k) in enumerate(zip(runs, ks)):
        C3, lab3 = out[r]
        X64 = X.astype(np.float64)
        lab_ref, sse_ref, _, _ = oracle.assign(X64, C3)
        assert np.array_equal(lab3, lab_ref), r
        assert abs(sse[r] - sse_ref) <= TOL * sse_ref, r
        assert iters[r] == 3
    # shadow step on the largest run at full k
    X, k = runs[2], ks[2]
    assert k * X.shape[1] > 4096
    shadow_steps(km, oracle, X, X[:k], steps=2)


@pytest.mark.parametrize("d", [8, 16])
def test_wide_narrow_rows_split_and_float32(km, oracle, d):
    """Runs of 8 or 16 attributes whose centers stream in chunks (k d > 4096,
    k up to 1500, not a multiple of 16): with 16-byte aligned rows the first
    distance pass runs on split bfloat16 matrix cores, with rows off that
    alignment on float32 ones.  Both give the same results bit for bit, every
    final label is the oracle's nearest center of the returned centers, and
    single moves of the largest run match the oracle's moves."""
    rng = np.random.default_rng(40 + d)
    runs, ks = [], []
    for j, n in enumerate([5000, 12000, 40000, 3001]):
        X, _ = synth.gaussian_blobs(n, d, int(rng.integers(4, 33)), seed=500 + 10 * d + j,
                                    sigma=(0.2, 1.5))
        runs.append(oracle.scale(X)[0])
        ks.append(int(min(-(-n // 4), 1500)) - 3 * j)
    assert all(k * d > 4096 for k in ks)
    out_a, it_a, sse_a = run_batch(km, runs, ks, 4, 0.0)
    out_m, it_m, sse_m = run_batch(km, runs, ks, 4, 0.0, pad=1)
    assert np.array_equal(it_a, it_m) and np.array_equal(sse_a, sse_m)
    for r, (X, k) in enumerate(zip(runs, ks)):
        assert np.array_equal(out_a[r][0], out_m[r][0]), r
        assert np.array_equal(out_a[r][1], out_m[r][1]), r
        lab_ref, sse_ref, _, _ = oracle.assign(X.astype(np.float64), out_a[r][0])
        assert np.array_equal(out_a[r][1], lab_ref), r
        assert abs(sse_a[r] - sse_ref) <= TOL * sse_ref, r
        assert it_a[r] == 4
    X, k = runs[1], ks[1]
    shadow_steps(km, oracle, X, X[:k], steps=2)


def test_forms_agree_on_large_k(km, oracle):
    rng = np.random.default_rng(44)
    runs, ks = [], []
    for j in range(4):
        n = int(rng.integers(3000, 8000))
        X, _ = synth.gaussian_blobs(n, 32, 12, seed=400 + j, sigma=0.5)
        runs.append(oracle.scale(X)[0])
        ks.append(300)
    a, ia, sa = run_batch(km, runs, ks, 8, 1e-6, form=0)
    b, ib, sb = run_batch(km, runs, ks, 8, 1e-6, form=1)
    assert np.array_equal(ia, ib) and np.array_equal(sa, sb)
    for (ca, la), (cb, lb) in zip(a, b):
        assert np.array_equal(ca, cb) and np.array_equal(la, lb)


# ------------------------------------------------ full-size workload, bench config
def _assign_chunked(oracle, S, C, chunk=1 << 16):
    """oracle.assign over all rows of S in chunks on a thread pool; the
    objective is summed in chunk order."""
    import concurrent.futures as cf
    C = np.asarray(C, np.float64)
    parts = [(a, min(a + chunk, S.shape[0])) for a in range(0, S.shape[0], chunk)]

    def one(ab):
        lab, sse, _, _ = oracle.assign(S[ab[0]:ab[1]].astype(np.float64), C)
        return lab, sse
    with cf.ThreadPoolExecutor(protocol.threads()) as ex:
        res = list(ex.map(one, parts))
    return np.concatenate([r[0] for r in res]), float(sum(r[1] for r in res))


def _golden_subclusters(name):
    """Digests of the oracle's scaling and subclustering of a full-size
    workload (tests/golden/make_fullsize_subclusters.py)."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "fullsize_subclusters.json")
    if not os.path.exists(path):
        return {"x": None}
    with open(path) as f:
        return json.load(f)[name]


def _digest(a):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.mark.timeout(900)
def test_mid_workload_full_size(km, oracle):
    """The benchmark's workload at full size (2^20 x 16, N = 8192, 256 local
    and 64 final centers, <= 30 moves or a move below 1e-6), through the
    same call the benchmark times, against the oracle:
    * scaling, subclusters (perm, offsets) bit-exact;
    * all 128 local runs: the oracle's own trajectory from the same start;
      every run without a near tie on that path must give the oracle's
      centers, objective and move count; every run passes the shadow step
      from the GPU's returned centers;
    * the final run: the oracle's final stage on the GPU's local centers
      (same protocol), and, when every local run agreed, the oracle's whole
      method on its own local centers;
    * labels and objective of all 2^20 points against the final centers."""
    job = synth.mid()
    n, d = job.X.shape
    out = km.cluster(dev(job.X), job.N, job.k_local, job.k_final, job.max_iter, job.tol,
                     intermediates=True, stats=True)
    S = host(out["S"])
    perm = host(out["perm"]).astype("<i8")
    gold = _golden_subclusters("mid")
    if _digest(job.X) == gold["x"]:
        # the oracle's own scaling and subclustering, by their digests
        assert _digest(S) == gold["s"]
        assert _digest(perm) == gold["perm"]
        Sr, permr = S, perm
        offr = np.append(np.arange(0, n, job.N, dtype=np.int64), n)
        assert _digest(offr.astype("<i8")) == gold["offsets"]
    else:
        Sr, _, _ = oracle.scale(job.X)
        assert np.array_equal(S, Sr)
        permr, offr, _ = oracle.subcluster(Sr, job.N)
        assert np.array_equal(perm, permr)
    T, k = len(offr) - 1, job.k_local
    st = out["stats"]
    assert st["T"] == T == 128 and st["M"] == T * k
    loc = host(out["local_centers"])
    lit = host(out["local_iters"])
    lsse = host(out["local_sse"])
    Ps = [Sr[permr[offr[t]:offr[t + 1]]] for t in range(T)]
    trajs = protocol.trajectories(oracle, [(P.astype(np.float64), P[:k]) for P in Ps],
                                  job.max_iter, job.tol)
    compared, agree = 0, 0
    for t in range(T):
        Ct = loc[t * k:(t + 1) * k]
        compared += protocol.check_independent(Ct, lsse[t], lit[t], trajs[t], job.tol, f"local {t}")
        agree += rel_err(Ct, trajs[t]["centers"]) <= TOL
    near = [t for t in range(T) if trajs[t]["min_margin"] <= protocol.NEAR_TIE]
    print(f"mid local runs: {compared} of {T} compared on independent trajectories, "
          f"{len(near)} with a near tie on the oracle's path, {agree} within 1e-5 of the oracle")
    assert compared + len(near) == T
    assert compared >= T // 2
    protocol.shadow(km, oracle, Ps, [loc[t * k:(t + 1) * k] for t in range(T)], what="mid local")

    # final run: the oracle's final stage from the GPU's local centers
    M = T * k
    stride = M // job.k_final
    fin = host(out["centers"])
    ftraj = protocol.trajectory(oracle, loc.astype(np.float64), loc[::stride][:job.k_final],
                                job.max_iter, job.tol)
    fcomp = protocol.check_independent(fin, None, st["final_iters"], ftraj, job.tol, "final")
    protocol.shadow(km, oracle, [loc], [fin], what="mid final")
    print(f"mid final run: {st['final_iters']} moves (oracle {ftraj['iters']}), "
          f"{'compared' if fcomp else 'near tie: shadow step only'}")
    if agree == T:
        # the whole method on the oracle's own local centers
        oloc = np.concatenate([tr["centers"] for tr in trajs])
        otraj = protocol.trajectory(oracle, oloc, oloc[::stride][:job.k_final], job.max_iter, job.tol)
        if otraj["min_margin"] > protocol.NEAR_TIE and ftraj["min_margin"] > protocol.NEAR_TIE:
            assert rel_err(fin, otraj["centers"]) <= TOL
            assert protocol.iters_agree(st["final_iters"], otraj, job.tol)

    # labels of all points and the objective
    lab, obj = _assign_chunked(oracle, Sr, fin)
    assert np.array_equal(host(out["labels"]), lab)
    assert abs(host(out["sse"])[0] - obj) <= TOL * obj


@pytest.mark.timeout(900)
def test_ragged_workload_full_size(km, oracle):
    """The ragged batch at full size (512 runs, n log-uniform in [1k, 64k],
    half d = 8 and half d = 32, k = min(ceil(n / 32), 1024), <= 30 moves or a
    move below 1e-6), every run scaled by the library and all of them in one
    batched call, as the benchmark times it:
    * every run's scaling bit-exact;
    * every run's labels equal the oracle's assignment against the run's
      returned centers, objective within 1e-5;
    * 48 sampled runs of up to 12k points (both d) against the oracle's own
      trajectories, per the comparison protocol;
    * the shadow step on those and on the 8 largest runs (k = 1024, more
      than 2^15 points: the runs beyond the on-chip budget)."""
    import concurrent.futures as cf
    rs = synth.ragged()
    Ss, parts, cinit, specs = [], [], [], []
    x_off = c_off = l_off = 0
    for X, k in zip(rs.X, rs.k):
        Sg, _, _ = km.scale(dev(X))
        n, d = Sg.shape
        Ss.append(Sg)
        parts.append(Sg.reshape(-1))
        cinit.append(Sg[:k].reshape(-1))
        specs.append((x_off, n, c_off, l_off, d, k))
        x_off += n * d
        c_off += k * d
        l_off += n
    C = torch.cat(cinit)
    lab = torch.empty(l_off, dtype=torch.int32, device="cuda:0")
    km.profile(True)
    it, sse = km.lloyd_batched(torch.cat(parts), specs, C, lab, rs.max_iter, rs.tol)
    Ch, lh, ih, sh = host(C), host(lab), host(it), host(sse)
    prof = km.profile_read()
    km.profile(False)
    # one call, both paths: the runs that fit on chip in the persistent
    # kernel, the others in per-phase launches
    assert prof["lloyd_fused"][0] >= 1 and prof["assign"][0] >= 1, prof
    with cf.ThreadPoolExecutor(protocol.threads()) as ex:
        Sr = list(ex.map(lambda X: oracle.scale(X)[0], rs.X))
    for j, Sg in enumerate(Ss):
        assert np.array_equal(host(Sg), Sr[j]), j
    del Ss, parts, cinit
    Cs = [Ch[co:co + k * d].reshape(k, d) for (xo, n, co, lo, d, k) in specs]
    labs = [lh[lo:lo + n] for (xo, n, co, lo, d, k) in specs]

    def assign_run(j):
        return oracle.assign(Sr[j].astype(np.float64), Cs[j])[:2]
    with cf.ThreadPoolExecutor(protocol.threads()) as ex:
        refs = list(ex.map(assign_run, range(len(specs))))
    for j, (lr, sr) in enumerate(refs):
        assert np.array_equal(labs[j], lr), j
        assert abs(sh[j] - sr) <= TOL * sr, j
        assert 1 <= ih[j] <= rs.max_iter, j
    ns = np.array([sp[1] for sp in specs])
    dd = np.array([sp[4] for sp in specs])
    rng = np.random.default_rng(8)
    sample = []
    for dv in (8, 32):
        pool = np.flatnonzero((dd == dv) & (ns <= 12000))
        sample += sorted(rng.choice(pool, 24, replace=False).tolist())
    trajs = protocol.trajectories(
        oracle, [(Sr[j].astype(np.float64), Sr[j][:rs.k[j]]) for j in sample], rs.max_iter, rs.tol)
    compared = sum(protocol.check_independent(Cs[j], sh[j], ih[j], tr, rs.tol, f"ragged run {j}")
                   for j, tr in zip(sample, trajs))
    print(f"ragged: {compared} of {len(sample)} sampled runs compared on independent trajectories")
    assert compared >= len(sample) // 2
    big = np.argsort(ns)[-8:].tolist()
    assert all(ns[j] > 1 << 15 and rs.k[j] == 1024 for j in big)
    assert any(dd[j] == 32 for j in big)
    shadow = sample + big
    protocol.shadow(km, oracle, [Sr[j] for j in shadow], [Cs[j] for j in shadow], what="ragged")


# ------------------------------------------- split-bfloat16 path (wide runs, BF16)
PREC_BF16 = 1


@pytest.mark.parametrize("n,d,k", [(3001, 32, 300), (2000, 48, 200), (1500, 64, 100), (900, 128, 300),
                                   (2600, 100, 257), (500, 128, 33), (2048, 128, 1024), (4100, 33, 130)])
def test_lloyd_shadow_bf16(km, oracle, n, d, k):
    """Split-bfloat16 products on matrix cores: labels must still be those of
    exact arithmetic, centers and objective within the tolerance, step by
    step against the oracle (attribute counts 32..128, padded and ragged
    tiles, k up to 1024)."""
    assert k * d > 4096
    X, _ = synth.gaussian_blobs(n, d, max(2, k // 8), seed=n + d + 1, sigma=0.7)
    S, _, _ = oracle.scale(X)
    shadow_steps(km, oracle, S, S[:k], steps=2, precision=PREC_BF16)


def test_lloyd_bf16_exact_ties(km, oracle):
    # every point equidistant from two copies of its center: exact ties on
    # every point, resolved to the lower index; the copies stay empty
    rng = np.random.default_rng(12)
    base = rng.uniform(0, 1, (40, 64)).astype(np.float32)
    X = np.repeat(base, 25, axis=0)
    C0 = np.concatenate([base, base])
    assert C0.shape[0] * 64 > 4096
    shadow_steps(km, oracle, X, C0, steps=2, precision=PREC_BF16)


def test_lloyd_bf16_dense_near_ties(km, oracle):
    # many centers packed inside one blob: small gaps, frequent two-way and
    # pooled rechecks
    X, _ = synth.gaussian_blobs(6000, 128, 2, seed=77, sigma=0.3)
    S, _, _ = oracle.scale(X)
    shadow_steps(km, oracle, S, S[:512], steps=2, precision=PREC_BF16)


def test_forms_agree_bf16(km, oracle):
    rng = np.random.default_rng(45)
    runs, ks = [], []
    for j in range(5):
        n = int(rng.integers(2000, 7000))
        d = [32, 64, 128, 40, 96][j]
        X, _ = synth.gaussian_blobs(n, d, 10, seed=500 + j, sigma=0.5)
        runs.append(oracle.scale(X)[0])
        ks.append(int(rng.integers(130, 600)))
    a, ia, sa = run_batch(km, runs, ks, 6, 1e-6, form=0, precision=PREC_BF16)
    b, ib, sb = run_batch(km, runs, ks, 6, 1e-6, form=1, precision=PREC_BF16)
    c, ic, sc = run_batch(km, runs, ks, 6, 1e-6, form=0, precision=PREC_BF16)
    f, i32, s32 = run_batch(km, runs, ks, 6, 1e-6, form=0, precision=0)
    assert np.array_equal(ia, ib) and np.array_equal(sa, sb) and np.array_equal(sa, sc)
    for (ca, la), (cb, lb), (cc, lc), (cf, lf) in zip(a, b, c, f):
        assert np.array_equal(ca, cb) and np.array_equal(la, lb)
        assert np.array_equal(ca, cc) and np.array_equal(la, lc)
        # exact labels in both precisions: the same trajectory
        assert np.array_equal(ca, cf) and np.array_equal(la, lf)
    assert np.array_equal(ia, i32) and np.array_equal(sa, s32)


def _keys(S, L):
    # the landmark key of Algorithm 1 in the oracle's arithmetic: binary64,
    # attributes left to right, separate multiply and add
    acc = np.zeros(S.shape[0])
    for j in range(S.shape[1]):
        q = S[:, j].astype(np.float64) - np.float64(L[j])
        acc = acc + q * q
    return acc


@pytest.mark.timeout(900)
def test_precision_workload_full_size(km, oracle):
    """The precision workload (n = 2^22, d = 128, N = 32768, 1024 local and
    256 final centers) through cluster() with split-bfloat16 products:
    scaling and the whole subclustering (perm of all 2^22 points) bit-exact
    against the oracle's, by the SHA-256 digests the oracle's own run wrote
    (its 128 rounds take minutes on one core; the oracle runs live only when
    the input differs from the one the digests were made from); sampled
    local runs and a sample of the final labels against the oracle."""
    import paper_1412_1947_amd as subkm
    job = synth.precision()
    n, d = job.X.shape
    gold = _golden_subclusters("precision")
    X = dev(job.X)
    out = km.cluster(X, job.N, job.k_local, job.k_final, job.max_iter, job.tol,
                     precision=subkm.PREC_BF16, intermediates=True, stats=True)
    S = host(out["S"])
    del X
    perm = host(out["perm"]).astype("<i8")
    N, T = job.N, out["stats"]["T"]
    assert T == n // N
    if _digest(job.X) == gold["x"]:
        assert _digest(S) == gold["s"]
        assert _digest(perm) == gold["perm"]
        assert _digest(np.arange(0, n + 1, N, dtype="<i8")) == gold["offsets"]
        Sr = S
    else:
        Sr, _, _ = oracle.scale(job.X)
        assert np.array_equal(S, Sr)
        permr, offr, _ = oracle.subcluster(Sr, N)
        assert np.array_equal(perm, permr)
    assert np.array_equal(np.sort(perm), np.arange(n))
    loc = host(out["local_centers"])
    lsse = host(out["local_sse"])
    lit = host(out["local_iters"])
    k = job.k_local
    sample = (0, T // 2, T - 1)
    Ps = [np.ascontiguousarray(Sr[perm[t * N:(t + 1) * N]]) for t in sample]
    Cs = [loc[t * k:(t + 1) * k] for t in sample]
    for t, P, C in zip(sample, Ps, Cs):
        _, obj, _, _ = oracle.assign(P.astype(np.float64), C)
        assert abs(lsse[t] - obj) <= TOL * obj
        assert 1 <= lit[t] <= job.max_iter
    # the shadow step of sampled local runs and of the final run, with
    # split-bfloat16 products: labels identical to binary64 arithmetic
    fin = host(out["centers"])
    protocol.shadow(km, oracle, Ps, Cs, precision=subkm.PREC_BF16, what="precision local")
    protocol.shadow(km, oracle, [loc], [fin], precision=subkm.PREC_BF16, what="precision final")
    # labels of all 2^22 points and the objective against the final centers
    lab, obj = _assign_chunked(oracle, Sr, fin)
    assert np.array_equal(host(out["labels"]), lab)
    assert abs(host(out["sse"])[0] - obj) <= TOL * obj


# ------------------------------------------------------------ memory and serving
@pytest.mark.parametrize("n,d,N,kl,kf,prec", [(4096, 4, 512, 32, 8, 0), (50000, 16, 8192, 256, 64, 0),
                                               (30000, 64, 8192, 256, 100, 0), (40000, 128, 8192, 512, 64, 1),
                                               (20000, 32, 4096, 256, 300, 1), (9000, 7, 1000, 90, 40, 0),
                                               (45000, 128, 8192, 256, 30, 1)])
def test_footprint_bounds_the_scratch(n, d, N, kl, kf, prec):
    """The footprint used for admission is an upper bound of the device memory
    a fresh context holds after the call (and not a wild over-estimate)."""
    import paper_1412_1947_amd as subkm
    X, _ = synth.gaussian_blobs(n, d, 20, seed=n + d, sigma=0.6)
    ctx = subkm.Context(0)
    try:
        ctx.cluster(dev(X), N, kl, kf, 8, 1e-6, precision=prec)
        torch.cuda.synchronize()
        used = ctx.device_bytes()
        fp = subkm.cluster_footprint(n, d, N, kl, kf)
        assert used <= fp, (used, fp)
        assert used >= fp // 4, (used, fp)
    finally:
        ctx.close()


def _serve_jobs():
    rng = np.random.default_rng(9)
    jobs = []
    for j, (n, d, kf, prec) in enumerate([(30000, 8, 40, 0), (5000, 4, 12, 0), (120000, 16, 64, 0),
                                          (60000, 64, 100, 0), (20000, 32, 200, 1), (45000, 128, 30, 1),
                                          (9000, 16, 8, 0), (70000, 4, 256, 0)]):
        X, _ = synth.gaussian_blobs(n, d, kf, seed=600 + j, sigma=0.5)
        jobs.append((torch.from_numpy(X).pin_memory(), kf, prec))
    return jobs


def _run_engine(eng, jobs, together):
    out = []
    if together:
        ids = [eng.submit(X, 8192, 256, kf, 30, 1e-6, precision=p) for X, kf, p in jobs]
        out = [eng.wait(i) for i in ids]
    else:
        for X, kf, p in jobs:
            out.append(eng.wait(eng.submit(X, 8192, 256, kf, 30, 1e-6, precision=p)))
    return out


def test_engine_alone_and_in_the_mix(km):
    """Every job gives the same result alone, in a mix of concurrent jobs, and
    through a direct cluster() call."""
    import paper_1412_1947_amd as subkm
    jobs = _serve_jobs()
    e1 = subkm.Engine(0, budget_bytes=64 << 30, slots=1)
    try:
        alone = _run_engine(e1, jobs, together=False)
    finally:
        e1.close()
    e4 = subkm.Engine(0, budget_bytes=64 << 30, slots=4)
    try:
        mix = _run_engine(e4, jobs, together=True)
    finally:
        e4.close()
    # the mix really overlapped: some job started before another finished
    spans = sorted((r["t_start"], r["t_done"]) for r in mix)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    for (X, kf, p), a, b in zip(jobs, alone, mix):
        assert a["sse"] == b["sse"]
        assert torch.equal(a["centers"], b["centers"]) and torch.equal(a["labels"], b["labels"])
        ref = km.cluster(dev(X.numpy()), 8192, 256, kf, 30, 1e-6, precision=p)
        assert host(ref["sse"])[0] == a["sse"]
        assert np.array_equal(host(ref["centers"]), a["centers"].numpy())
        assert np.array_equal(host(ref["labels"]), a["labels"].numpy())


def test_engine_budget_admission():
    """Jobs are admitted only while the engine stays within its budget: with
    room for one job of a kind at a time, such jobs run one after the other;
    a mix never holds more than the budget; a job larger than the budget is
    refused at submission."""
    import paper_1412_1947_amd as subkm
    same = []
    for j in range(4):
        X, _ = synth.gaussian_blobs(40000, 16, 32, seed=700 + j, sigma=0.5)
        same.append((torch.from_numpy(X).pin_memory(), 32, 0))
    fp = subkm.job_footprint(40000, 16, 8192, 256, 32)
    eng = subkm.Engine(0, budget_bytes=int(fp * 1.5), slots=4)
    try:
        res = _run_engine(eng, same, together=True)
        spans = sorted((r["t_start"], r["t_done"]) for r in res)
        for i in range(len(spans) - 1):
            assert spans[i + 1][0] >= spans[i][1], spans
        for r in res:
            assert r["device_bytes"] <= fp * 1.5
    finally:
        eng.close()
    jobs = _serve_jobs()
    budget = int(max(subkm.job_footprint(X.shape[0], X.shape[1], 8192, 256, kf) for X, kf, _ in jobs) * 1.2)
    eng = subkm.Engine(0, budget_bytes=budget, slots=4)
    try:
        res = _run_engine(eng, jobs, together=True)
        for r in res:
            assert r["slot_bytes_after"] <= r["slot_bytes_admitted"], r
            assert r["device_bytes"] <= budget
        big = torch.zeros((400000, 64), dtype=torch.float32)
        with pytest.raises(subkm.SubkmError):
            eng.submit(big, 8192, 256, 64, 30, 1e-6)
    finally:
        eng.close()


# ------------------------------------------------- direct Lloyd (comparison baseline)
def test_direct_lloyd_full_size(km, oracle):
    """Lloyd on all 2^20 points of the benchmark workload at once (the
    paper's comparison baseline): one run far beyond the blocks that can
    share partial sums, so it takes the wide path.  One move from the
    strided start against the oracle; the plain form gives the same bits."""
    job = synth.mid()
    S, _, _ = oracle.scale(job.X)
    n, d = S.shape
    k = job.k_final
    C0 = S[np.arange(k) * (n // k)]
    shadow_steps(km, oracle, S, C0, steps=1)
    a, ia, sa = run_batch(km, [S], [k], 3, 0.0, form=0)
    b, ib, sb = run_batch(km, [S], [k], 3, 0.0, form=1)
    assert np.array_equal(sa, sb) and np.array_equal(a[0][0], b[0][0])


# ------------------------------------------------- the paper's 2-D workload shape
@pytest.mark.timeout(600)
def test_paper2d_direct_full_size(km, oracle):
    """Lloyd on all 500,000 points of the 2-D, 500-points-per-cluster
    workload with 1000 centers (the traditional side of the timing
    experiment): one move from the strided start against the oracle."""
    X = synth.paper2d(500_000)
    S, _, _ = oracle.scale(X)
    k = 1000
    shadow_steps(km, oracle, S, S[np.arange(k) * (len(S) // k)], steps=1)


@pytest.mark.parametrize("scheme", [0, 1])
def test_paper2d_two_level_scaled_down(km, oracle, scheme):
    """The two-level method at the sweep's shape, scaled down so that the
    oracle finishes: 2-D blobs, 500 points per cluster, compression 5."""
    import paper_1412_1947_amd as pkg
    X = synth.paper2d(20_000)
    N, c, kf = 2000, 5, 40
    out = km.cluster(dev(X), N, N // c, kf, 30, 1e-6, intermediates=True, stats=True,
                     scheme=scheme)
    ref = oracle.cluster(X, N, N // c, kf, 30, 1e-6, scheme=scheme)
    assert out["stats"]["M"] == ref["M"]
    assert np.array_equal(host(out["perm"]), ref["perm"])
    assert rel_err(host(out["local_centers"])[:ref["M"]], ref["local_centers"]) <= TOL
    assert rel_err(host(out["centers"]), ref["centers"]) <= TOL
    assert abs(host(out["sse"])[0] - ref["sse"]) <= TOL * ref["sse"]
