"""The allocation-free scaling entry point (subkm_scale_noalloc), called
through the C ABI: the same bits as subkm_scale on two calls in a row, the
second with a smaller input, for the narrow and the wide form of the min/max
pass (the widest rows run with a capped grid), non-finite input refused, and
the calling context's scratch left empty."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _call(L, ctx, X, S, mins, maxs):
    n, d = X.shape
    P = ctypes.c_void_p
    return L.subkm_scale_noalloc(ctx._h, P(X.data_ptr()), n, d, P(S.data_ptr()),
                                 P(mins.data_ptr()), P(maxs.data_ptr()))


@pytest.mark.parametrize("shapes", [[(300_000, 16), (1_000, 16)], [(200_000, 130), (777, 130)],
                                    [(3_000, 4096), (65, 4096)], [(70_001, 3), (2, 3)]])
def test_scale_noalloc_matches_scale(oracle, shapes):
    import paper_1412_1947_amd as pkg
    L = pkg.lib()
    fresh = pkg.Context(0)   # only the allocation-free call runs on it
    ref = pkg.Context(0)     # the allocating entry point, for comparison
    try:
        for j, (n, d) in enumerate(shapes):
            rng = np.random.default_rng(n + d)
            Xh = (rng.standard_normal((n, d)) * rng.uniform(0.1, 50, d) + rng.uniform(-5, 5, d)).astype(np.float32)
            if d > 2:
                Xh[:, 1] = 0.25  # constant attribute
            X = torch.from_numpy(Xh).to("cuda:0")
            S = torch.full((n, d), np.nan, dtype=torch.float32, device="cuda:0")
            mins = torch.full((d,), np.nan, dtype=torch.float32, device="cuda:0")
            maxs = torch.full((d,), np.nan, dtype=torch.float32, device="cuda:0")
            torch.cuda.synchronize()
            print(f"scale_noalloc call {j}: n={n} d={d}", flush=True)
            assert _call(L, fresh, X, S, mins, maxs) == 0, L.subkm_last_error(fresh._h)
            Sr, mnr, mxr = ref.scale(X)
            torch.cuda.synchronize()
            assert torch.equal(S, Sr) and torch.equal(mins, mnr) and torch.equal(maxs, mxr)
            So, mno, mxo = oracle.scale(Xh)
            assert np.array_equal(S.cpu().numpy(), So)
            assert np.array_equal(mins.cpu().numpy(), mno) and np.array_equal(maxs.cpu().numpy(), mxo)
        assert fresh.device_bytes() == 0
    finally:
        fresh.close()
        ref.close()


def test_scale_noalloc_refuses_non_finite():
    import paper_1412_1947_amd as pkg
    L = pkg.lib()
    ctx = pkg.Context(0)
    try:
        for bad in (np.nan, np.inf):
            Xh = np.ones((5000, 8), np.float32)
            Xh[1234, 5] = bad
            X = torch.from_numpy(Xh).to("cuda:0")
            S = torch.empty_like(X)
            mins = torch.empty(8, dtype=torch.float32, device="cuda:0")
            maxs = torch.empty(8, dtype=torch.float32, device="cuda:0")
            torch.cuda.synchronize()
            assert _call(L, ctx, X, S, mins, maxs) == 1
            assert b"NaN" in L.subkm_last_error(ctx._h)
        # a clean call after the refused ones: the flag was cleared
        Xh = np.arange(40, dtype=np.float32).reshape(10, 4)
        X = torch.from_numpy(Xh).to("cuda:0")
        S = torch.empty_like(X)
        mins = torch.empty(4, dtype=torch.float32, device="cuda:0")
        maxs = torch.empty(4, dtype=torch.float32, device="cuda:0")
        assert _call(L, ctx, X, S, mins, maxs) == 0
        torch.cuda.synchronize()
        assert np.array_equal(mins.cpu().numpy(), Xh.min(axis=0))
        assert ctx.device_bytes() == 0
    finally:
        ctx.close()
