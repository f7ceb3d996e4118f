"""Pins of the oracle's 3D grids (Sec. 3.1 extended by one axis) against facts
built without its 3D code: Kronecker products of 1D matrices (np.kron), the
degenerate shapes that are 1D and 2D grids, explicit integer products, and
brute-force four-index sums in rational arithmetic."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import gw_oracle as O
from paper_2404_08970_amd import inputs


def _d1(n, m):
    i = np.arange(n, dtype=np.int64)
    d = np.abs(i[:, None] - i[None, :])
    return np.ones((n, n), dtype=np.int64) if m == 0 else d ** m


@pytest.mark.parametrize("shape,k", [((2, 3, 4), 1), ((3, 2, 2), 2), ((2, 2, 3), 3), ((4, 1, 3), 2)])
def test_l1pow_distance_is_kronecker_sum(shape, k):
    D0, H, W = shape
    ref = np.zeros((D0 * H * W,) * 2, dtype=np.int64)
    for a in range(k + 1):
        for b in range(k + 1 - a):
            c = k - a - b
            coef = math.factorial(k) // (math.factorial(a) * math.factorial(b) * math.factorial(c))
            ref += coef * np.kron(np.kron(_d1(D0, a), _d1(H, b)), _d1(W, c))
    got = O.integer_distance(O.Grid(shape, 1.0, k))
    assert np.array_equal(got, ref)


def test_sqeuclid_distance_is_kronecker_sum():
    D0, H, W = 3, 4, 2
    ref = (np.kron(np.kron(_d1(D0, 2), _d1(H, 0)), _d1(W, 0))
           + np.kron(np.kron(_d1(D0, 0), _d1(H, 2)), _d1(W, 0))
           + np.kron(np.kron(_d1(D0, 0), _d1(H, 0)), _d1(W, 2)))
    got = O.integer_distance(O.Grid((D0, H, W), 1.0, 2, O.METRIC_SQEUCLID))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("k,metric", [(1, O.METRIC_L1POW), (3, O.METRIC_L1POW), (2, O.METRIC_SQEUCLID)])
def test_degenerate_shapes_are_lower_dimensional_grids(k, metric):
    assert np.array_equal(O.integer_distance(O.Grid((1, 4, 5), 1.0, k, metric)),
                          O.integer_distance(O.Grid((4, 5), 1.0, k, metric)))
    if metric == O.METRIC_L1POW:
        assert np.array_equal(O.integer_distance(O.Grid((1, 1, 7), 1.0, k)),
                              O.integer_distance(O.Grid((7,), 1.0, k)))


def test_rows_match_full_matrix():
    g = O.Grid((3, 4, 5), 0.5, 2)
    rows = np.array([0, 7, 33, 59])
    assert np.array_equal(O.integer_distance_rows(g, rows), O.integer_distance(g)[rows])


@pytest.mark.parametrize("shape,k,metric", [((3, 4, 5), 1, O.METRIC_L1POW), ((2, 3, 3), 4, O.METRIC_L1POW),
                                            ((4, 2, 3), 2, O.METRIC_SQEUCLID)])
def test_grid_apply_is_the_integer_product(shape, k, metric):
    g = O.Grid(shape, 1.0, k, metric)
    rng = inputs.rng_for(920, k)
    X = rng.integers(-20, 21, size=(g.size, 3)).astype(np.float64)
    ref = O.integer_distance(g) @ X.astype(np.int64)
    assert np.array_equal(O.grid_apply(g, X), ref.astype(np.float64))


CASES = [(O.Grid((2, 2, 2), 0.5, 1), O.Grid((3,), 0.25, 2)),
         (O.Grid((2, 1, 3), 0.25, 2, O.METRIC_SQEUCLID), O.Grid((2, 3), 0.5, 1))]


@pytest.mark.parametrize("gx,gy", CASES)
def test_grad_equals_four_index_sum(gx, gy):
    rng = inputs.rng_for(921, gx.size, gy.size)
    T = rng.integers(0, 16, size=(gx.size, gy.size)) / 32.0
    p, q = T.sum(axis=1), T.sum(axis=0)
    hx = Fraction(gx.h) ** (2 if gx.metric == O.METRIC_SQEUCLID else gx.k)
    hy = Fraction(gy.h) ** (2 if gy.metric == O.METRIC_SQEUCLID else gy.k)
    DX, DY = O.integer_distance(gx), O.integer_distance(gy)
    M, N = T.shape
    Tf = [[Fraction(float(T[j, c])) for c in range(N)] for j in range(M)]
    ref = np.zeros((M, N))
    for i in range(M):
        for a in range(N):
            s = Fraction(0)
            for j in range(M):
                for c in range(N):
                    d = hx * int(DX[i, j]) - hy * int(DY[a, c])
                    s += d * d * Tf[j][c]
            ref[i, a] = float(s)
    for G in (O.grad_dense(gx, gy, p, q, T), O.grad_pascal(gx, gy, p, q, T)):
        assert np.max(np.abs(G - ref)) <= 1e-14 * np.max(np.abs(ref))
