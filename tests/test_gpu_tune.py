"""The schedule tuner of the batched Lloyd form: tuned and untuned calls give
the same bits (the schedule only moves work between blocks: sums are exact
integers, labels exact), the caller's starting centers survive the tuning
runs, and tuned schedules round-trip through a file.
"""
import os

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _cluster(ctx, job):
    return ctx.cluster(dev(job.X), job.N, job.k_local, job.k_final, job.max_iter, job.tol,
                       intermediates=True)


def test_tuned_cluster_same_bits(tmp_path):
    import paper_1412_1947_amd as pkg
    job = synth.mid(n=1 << 17)
    job = synth.ClusterJob(job.X, 8192, 256, 64, 12, 1e-6)
    plain = pkg.Context(0)
    ref = _cluster(plain, job)
    tuned = pkg.Context(0)
    tuned.tune(True)
    for _ in range(2):  # first call tunes, second uses the tuned schedules
        out = _cluster(tuned, job)
        for key in ("local_centers", "local_iters", "centers", "labels", "sse"):
            assert np.array_equal(host(out[key]), host(ref[key])), key
    assert tuned.tuned() == 2  # the local runs and the final run
    path = os.path.join(tmp_path, "sched.txt")
    tuned.tune_save(path)
    other = pkg.Context(0)
    other.tune_load(path)
    assert other.tuned() == 2
    out = _cluster(other, job)  # tuning off: the loaded schedules are used
    assert other.tuned() == 2
    assert np.array_equal(host(out["centers"]), host(ref["centers"]))
    for c in (plain, tuned, other):
        c.close()


def test_tuning_restores_the_callers_centers():
    import paper_1412_1947_amd as pkg
    rng = np.random.default_rng(9)
    runs, C0, Xs, off, coff = [], [], [], 0, 0
    for r in range(6):
        n, d, k = 3000 + 500 * r, 8, 40
        X = rng.uniform(0, 1, (n, d)).astype(np.float32)
        Xs.append(X)
        C0.append(X[rng.choice(n, k, replace=False)])
        runs.append((off * d, n, coff * d, off, d, k))
        off += n
        coff += k
    P = dev(np.concatenate(Xs))
    Cs = np.concatenate(C0)
    ctxs = [pkg.Context(0), pkg.Context(0)]
    ctxs[1].tune(True)
    res = []
    for ctx in ctxs:
        C = dev(Cs)
        lab = torch.empty(off, dtype=torch.int32, device="cuda:0")
        it, sse = ctx.lloyd_batched(P.reshape(-1), runs, C, lab, 15, 0.0)
        res.append((host(C), host(lab), host(it), host(sse)))
    assert ctxs[1].tuned() == 1
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)
    for c in ctxs:
        c.close()


def test_tune_load_rejects_malformed(tmp_path):
    import paper_1412_1947_amd as pkg
    path = os.path.join(tmp_path, "bad.txt")
    with open(path, "w") as f:
        f.write("not a schedule file\n")
    ctx = pkg.Context(0)
    with pytest.raises(pkg.SubkmError):
        ctx.tune_load(path)
    with open(path, "w") as f:
        f.write("subkm-tune 1\n1 2 3 4 5 0 1 0.5\n")  # block cap 0
    with pytest.raises(pkg.SubkmError):
        ctx.tune_load(path)
    with open(path, "w") as f:
        f.write("subkm-tune 2\n1 2 3 4 5 64 1 0 0.5\n")  # no tiles per block
    with pytest.raises(pkg.SubkmError):
        ctx.tune_load(path)
    with open(path, "w") as f:
        f.write("subkm-tune 2\n1 2 3 4 5 64 1 0.5\n")  # a field missing
    with pytest.raises(pkg.SubkmError):
        ctx.tune_load(path)
    with open(path, "w") as f:
        f.write("subkm-tune 3\n1 2 3 4 5 64 1 2 0.5\n")  # no exchange field
    with pytest.raises(pkg.SubkmError):
        ctx.tune_load(path)
    with open(path, "w") as f:
        f.write("subkm-tune 3\n1 2 3 4 5 64 1 2 2 0.5\n")  # unknown exchange
    with pytest.raises(pkg.SubkmError):
        ctx.tune_load(path)
    # the earlier formats (no exchange field; nor a tiles field) still load
    with open(path, "w") as f:
        f.write("subkm-tune 1\n1 2 3 4 5 64 1 0.5\n")
    ctx.tune_load(path)
    assert ctx.tuned() == 1
    with open(path, "w") as f:
        f.write("subkm-tune 2\n1 2 3 4 5 64 1 2 0.5\n2 2 3 4 5 64 1 1 0.5\n")
    ctx.tune_load(path)
    assert ctx.tuned() == 2
    with open(path, "w") as f:
        f.write("subkm-tune 3\n3 2 3 4 5 64 1 2 1 0.5\n")
    ctx.tune_load(path)
    assert ctx.tuned() == 3
    ctx.close()


def _shape_line(runs, precision, sched):
    """A schedule-file entry for the shape of `runs` (see the tuner's key:
    runs, points, smallest and largest d and k, precision and moves)."""
    n = sum(r[1] for r in runs)
    ds = [r[4] for r in runs]
    ks = [r[5] for r in runs]
    v = [len(runs), n, (min(ds) << 32) | max(ds), (min(ks) << 32) | max(ks), (precision << 1) | 1]
    return " ".join("%x" % x for x in v) + " %d %d %d %d 1.0\n" % sched


@pytest.mark.parametrize("shape", ["one_run", "many_runs"])
def test_every_exchange_mode_same_bits(tmp_path, shape):
    """Forced schedules, both per-move exchanges (published parts with slice
    sums; shared totals with integer atomics) and several blocks-per-run
    caps, give the bits of the default schedule: centers, labels, moves and
    objectives."""
    import paper_1412_1947_amd as pkg
    rng = np.random.default_rng(21)
    if shape == "one_run":
        # one run of a final stage's shape: many blocks share every move
        specs = [(32768, 16, 64)]
    else:
        specs = [(6000 + 700 * r, 16, 48 + 16 * (r % 3)) for r in range(12)]
    runs, Xs, C0, off, coff = [], [], [], 0, 0
    for n, d, k in specs:
        means = rng.normal(0, 3, (k, d))
        X = (means[rng.integers(0, k, n)] + rng.normal(0, 1, (n, d))).astype(np.float32)
        X = (X - X.min(0)) / (X.max(0) - X.min(0))
        Xs.append(X.astype(np.float32))
        C0.append(X[rng.choice(n, k, replace=False)])
        runs.append((off * d, n, coff * d, off, d, k))
        off += n
        coff += k
    P = dev(np.concatenate(Xs))
    Cs = np.concatenate(C0)
    # k_final-sized runs reach the split path in FP32 at d = 16
    prec = pkg.PREC_FP32

    def run(ctx):
        C = dev(Cs)
        lab = torch.empty(off, dtype=torch.int32, device="cuda:0")
        it, sse = ctx.lloyd_batched(P.reshape(-1), runs, C, lab, 20, 0.0, prec)
        return host(C), host(lab), host(it), host(sse)

    base = pkg.Context(0)
    ref = run(base)
    base.close()
    assert int(ref[2].min()) >= 2  # every run moves: the exchange runs
    for sched in [(128, 1, 1, 0), (128, 1, 1, 1), (64, 1, 2, 1), (16, 1, 2, 1), (4, 1, 2, 1),
                  (2, 1, 1, 1)]:
        path = os.path.join(tmp_path, "s.txt")
        with open(path, "w") as f:
            f.write("subkm-tune 3\n" + _shape_line(runs, prec, sched))
        ctx = pkg.Context(0)
        ctx.tune_load(path)
        assert ctx.tuned() == 1
        got = run(ctx)
        assert ctx.tuned() == 1  # the loaded schedule served the call
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), sched
        ctx.close()
