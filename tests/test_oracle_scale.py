"""Pins of the oracle's min-max feature scaling (Sec. II, Algorithm 1 step 1).

Each check is fixed by the mathematics of min-max scaling, not by the
oracle's own formula: exact end points, range, monotonicity, invariance under
exact affine maps, a hand-worked closed form, and rejection of non-finite
input.
"""
import numpy as np
import pytest

import synth


def test_closed_form_small(oracle):
    # attribute 0: {0,4,2,1,3} -> x/4 exactly; attribute 1 constant -> 0;
    # attribute 2: {-2,-1,0,1,2} -> (x+2)/4
    X = np.array([[0, 7, -2], [4, 7, -1], [2, 7, 0], [1, 7, 1], [3, 7, 2]], np.float32)
    S, mn, mx = oracle.scale(X)
    np.testing.assert_array_equal(mn, [0, 7, -2])
    np.testing.assert_array_equal(mx, [4, 7, 2])
    np.testing.assert_array_equal(S[:, 0], [0, 1, 0.5, 0.25, 0.75])
    np.testing.assert_array_equal(S[:, 1], 0)
    np.testing.assert_array_equal(S[:, 2], [0, 0.25, 0.5, 0.75, 1])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_endpoints_range_monotone(oracle, seed):
    rng = np.random.default_rng(seed)
    X = (rng.standard_normal((777, 9)) * rng.uniform(0.1, 1e3, 9) + rng.uniform(-50, 50, 9)).astype(np.float32)
    X[:, 4] = 3.25  # constant attribute
    S, mn, mx = oracle.scale(X)
    for j in range(9):
        col = S[:, j]
        if j == 4:
            assert np.all(col == 0.0)
            continue
        assert col.min() == 0.0 and col.max() == 1.0
        assert col[np.argmin(X[:, j])] == 0.0 and col[np.argmax(X[:, j])] == 1.0
        o = np.argsort(X[:, j], kind="stable")
        assert np.all(np.diff(col[o]) >= 0)  # monotone in the raw value
    assert np.all((S >= 0) & (S <= 1))
    np.testing.assert_array_equal(mn, X.min(0))
    np.testing.assert_array_equal(mx, X.max(0))


def test_exact_affine_invariance(oracle):
    # scaling by a power of two and shifting by a value that keeps every
    # difference exact leave min-max scaled data bit-for-bit unchanged
    X = synth.tiny().X
    S, _, _ = oracle.scale(X)
    S2, _, _ = oracle.scale(X * np.float32(8.0))
    np.testing.assert_array_equal(S, S2)
    Xi = np.round(X * 64).astype(np.float32)  # values on a 1/64 grid
    A, _, _ = oracle.scale(Xi)
    B, _, _ = oracle.scale(Xi + np.float32(1024.0))
    np.testing.assert_array_equal(A, B)


def test_reflection(oracle):
    # scale(-X) = 1 - scale(X) up to one rounding of each side
    X = synth.tiny().X
    S, _, _ = oracle.scale(X)
    R, _, _ = oracle.scale(-X)
    assert np.max(np.abs(R.astype(np.float64) - (1.0 - S.astype(np.float64)))) <= 2 ** -23


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_rejects_non_finite(oracle, bad):
    X = np.ones((5, 3), np.float32)
    X[2, 1] = bad
    with pytest.raises(ValueError):
        oracle.scale(X)
