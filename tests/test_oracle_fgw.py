"""Pins of the oracle's fused GW (Remark, Entropic algorithm for FGW) against
facts that do not come from the oracle itself: exact four-index sums in
rational arithmetic for the gradient and the objective, the reduction to GW at
theta = 1, and at theta = 0 the Gibbs form and marginals of the entropic OT
plan of the fixed cost C o C."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import gw_oracle as O
from paper_2404_08970_amd import inputs


def _frac_grid_matrix(g):
    hk = Fraction(g.h) ** (2 if g.metric == O.METRIC_SQEUCLID else g.k)
    Di = O.integer_distance(g)
    return [[hk * int(Di[i, j]) for j in range(Di.shape[1])] for i in range(Di.shape[0])]


CASES = [
    (O.Grid((5,), 0.25, 1), O.Grid((4,), 0.5, 2)),
    (O.Grid((2, 3), 0.5, 1), O.Grid((3, 2), 0.25, 2)),
    (O.Grid((2, 2), 0.5, 2, O.METRIC_SQEUCLID), O.Grid((5,), 0.25, 1)),
]
THETA = Fraction(3, 8)  # dyadic: exact in binary floating point


def _dyadic_case(gx, gy, key):
    rng = inputs.rng_for(700, key, gx.size, gy.size)
    T = rng.integers(0, 32, size=(gx.size, gy.size)) / 64.0
    fa = rng.integers(-8, 9, size=gx.size) / 4.0
    fb = rng.integers(-8, 9, size=gy.size) / 4.0
    return T, fa, fb


@pytest.mark.parametrize("gx,gy", CASES)
def test_grad_fgw_equals_four_index_sum(gx, gy):
    """[grad E_fgw]_ip / 2 = (1 - theta)/2 c_ip^2 + theta sum_jq (dX_ij - dY_pq)^2 T_jq."""
    T, fa, fb = _dyadic_case(gx, gy, 1)
    p, q = T.sum(axis=1), T.sum(axis=0)  # the decomposition uses T's own marginals
    DX, DY = _frac_grid_matrix(gx), _frac_grid_matrix(gy)
    M, N = T.shape
    Tf = [[Fraction(float(T[j, k])) for k in range(N)] for j in range(M)]
    ref = np.zeros((M, N))
    for i in range(M):
        for pp in range(N):
            s = Fraction(0)
            for j in range(M):
                for k in range(N):
                    d = DX[i][j] - DY[pp][k]
                    s += d * d * Tf[j][k]
            c = Fraction(float(fa[i])) - Fraction(float(fb[pp]))
            ref[i, pp] = float((1 - THETA) / 2 * c * c + THETA * s)
    G = O.grad_fgw(gx, gy, p, q, T, fa, fb, float(THETA))
    assert np.max(np.abs(G - ref)) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("gx,gy", CASES)
def test_objective_fgw_equals_four_index_sum(gx, gy):
    T, fa, fb = _dyadic_case(gx, gy, 2)
    DX, DY = _frac_grid_matrix(gx), _frac_grid_matrix(gy)
    M, N = T.shape
    Tf = [[Fraction(float(T[i, k])) for k in range(N)] for i in range(M)]
    quad = Fraction(0)
    lin = Fraction(0)
    for i in range(M):
        for pp in range(N):
            if Tf[i][pp] == 0:
                continue
            c = Fraction(float(fa[i])) - Fraction(float(fb[pp]))
            lin += c * c * Tf[i][pp]
            for j in range(M):
                for k in range(N):
                    d = DX[i][j] - DY[pp][k]
                    quad += d * d * Tf[i][pp] * Tf[j][k]
    ref = float((1 - THETA) * lin + THETA * quad)
    got, _ = O.objective_fgw(gx, gy, T, fa, fb, float(THETA), 0.01)
    assert abs(got - ref) <= 1e-14 * abs(ref)


def test_theta_one_is_gw():
    gx, gy = O.Grid((12,), 1 / 11, 2), O.Grid((9,), 1 / 8, 1)
    rng = inputs.rng_for(701)
    p, q = inputs.dirichlet(12, rng), inputs.dirichlet(9, rng)
    fa, fb = rng.normal(size=12), rng.normal(size=9)
    T0, f0, g0, o0 = O.solve(gx, gy, p, q, 0.05, 3, 20)
    T1, f1, g1, o1 = O.solve_fgw(gx, gy, p, q, fa, fb, 1.0, 0.05, 3, 20)
    assert np.array_equal(T0, T1) and np.array_equal(f0, f1) and np.array_equal(g0, g1)
    assert o0 == o1


def test_gradient_is_affine_in_theta():
    gx, gy = O.Grid((7,), 1 / 6, 1), O.Grid((6,), 1 / 5, 2)
    rng = inputs.rng_for(702)
    T = inputs.random_plan(7, 6, rng)
    p, q = T.sum(axis=1), T.sum(axis=0)
    fa, fb = rng.normal(size=7), rng.normal(size=6)
    g1 = O.grad_fgw(gx, gy, p, q, T, fa, fb, 1.0)
    g0 = O.grad_fgw(gx, gy, p, q, T, fa, fb, 0.0)
    gt = O.grad_fgw(gx, gy, p, q, T, fa, fb, 0.3)
    assert np.allclose(gt, 0.3 * g1 + 0.7 * g0, rtol=1e-13, atol=1e-15)
    assert np.allclose(g1, O.grad_dense(gx, gy, p, q, T), rtol=0, atol=0)
    assert np.allclose(g0, 0.5 * O.feature_cost_sq(fa, fb), rtol=0, atol=0)


def test_theta_zero_is_entropic_ot_of_feature_cost():
    """theta = 0: the cost C o C does not depend on T, so every outer step
    returns the entropic OT plan of C o C.  Checked without the oracle's
    Sinkhorn: the plan has the Gibbs form T_ip = a_i b_p exp(-c_ip^2 / eps)
    (log T + c^2/eps has zero mixed second differences), its column sums are q
    (the last update is on g) and its row sums approach p."""
    gx, gy = O.Grid((10,), 1 / 9, 1), O.Grid((8,), 1 / 7, 1)
    rng = inputs.rng_for(703)
    p, q = inputs.dirichlet(10, rng), inputs.dirichlet(8, rng)
    fa, fb = np.linspace(0, 1, 10), np.linspace(0, 1, 8) ** 2
    eps = 0.05
    T, f, g, _ = O.solve_fgw(gx, gy, p, q, fa, fb, 0.0, eps, 3, 400)
    L = np.log(T) + O.feature_cost_sq(fa, fb) / eps
    mixed = L[1:, 1:] - L[1:, :-1] - L[:-1, 1:] + L[:-1, :-1]
    assert np.max(np.abs(mixed)) <= 1e-9
    assert np.max(np.abs(T.sum(axis=0) - q)) <= 1e-14
    assert np.max(np.abs(T.sum(axis=1) - p)) <= 1e-10
