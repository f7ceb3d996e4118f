"""Pins of the oracle's unbalanced GW (Remark, Entropic algorithm for UGW)
against facts outside its own arithmetic: the quadratic-KL identity by brute
force over product measures, the marginal relation of the unbalanced Sinkhorn
potentials, the closed-form plan of a zero cost, the balanced limit rho -> inf
(pinned balanced oracle), and the divergence by explicit four-index sums."""
import math

import numpy as np
import pytest

from oracle import gw_oracle as O
from paper_2404_08970_amd import inputs


def _kl_brute(a, b):
    s = 0.0
    for x, y in zip(a.ravel(), b.ravel()):
        if x > 0:
            s += x * math.log(x / y)
    return s - a.sum() + b.sum()


def test_quad_kl_identity_by_brute_force():
    rng = inputs.rng_for(940)
    a = rng.uniform(0.1, 2.0, 7)
    b = rng.uniform(0.1, 2.0, 7)
    a[2] = 0.0
    brute = _kl_brute(np.outer(a, a), np.outer(b, b))
    assert abs(O.quad_kl(a, b) - brute) <= 1e-12 * abs(brute)


def test_uot_column_marginal_relation():
    """After the g update, column p of the plan sums to v_p exp(-g_p / rho)."""
    rng = inputs.rng_for(941)
    C = rng.uniform(0, 1, (9, 7))
    u, v = rng.uniform(0.5, 1.5, 9), rng.uniform(0.5, 1.5, 7)
    u[4] = 0.0
    rho, eps = 0.7, 0.05
    for iters in (1, 3, 20):
        f, g = O.uot_sinkhorn(C, u, v, rho, eps, iters)
        P = O.uot_plan(C, f, g, u, v, eps)
        assert np.allclose(P.sum(axis=0), v * np.exp(-g / rho), rtol=1e-12, atol=0)
        assert np.all(P[4] == 0.0)


def test_uot_zero_cost_closed_form():
    """C = 0: the optimum is t u (x) v with t = (m(u) m(v))^(-rho / (2 rho + eps))
    (minimise 2-sided KL plus entropy over the scale t)."""
    rng = inputs.rng_for(942)
    u, v = rng.uniform(0.2, 1.0, 6), rng.uniform(0.5, 3.0, 5)
    rho, eps = 0.4, 0.1
    f, g = O.uot_sinkhorn(np.zeros((6, 5)), u, v, rho, eps, 400)
    P = O.uot_plan(np.zeros((6, 5)), f, g, u, v, eps)
    t = (u.sum() * v.sum()) ** (-rho / (2 * rho + eps))
    assert np.allclose(P, t * np.outer(u, v), rtol=1e-10, atol=0)


def test_uot_balanced_limit():
    rng = inputs.rng_for(943)
    C = rng.uniform(0, 1, (10, 8))
    p, q = inputs.dirichlet(10, rng), inputs.dirichlet(8, rng)
    eps = 0.1
    f, g = O.uot_sinkhorn(C, p, q, 1e9, eps, 3000)
    P = O.uot_plan(C, f, g, p, q, eps)
    fb, gb = O.sinkhorn(C, p, q, eps, 3000)
    Pb = O.plan(C, fb, gb, eps)
    assert np.max(np.abs(P - Pb)) <= 1e-7 * np.max(Pb)


def test_solve_ugw_balanced_limit_is_gw():
    """rho -> inf with balanced marginals: each UGW step minimises
    <G, T> + eps KL(T|u (x) v) over the couplings, the GW mirror-descent step
    <2G, T> + eps' H(T) with eps' = 2 eps (the KL reference only shifts the
    potentials on couplings)."""
    gx, gy = O.Grid((9,), 1 / 8, 1), O.Grid((7,), 1 / 6, 2)
    rng = inputs.rng_for(944)
    p, q = inputs.dirichlet(9, rng), inputs.dirichlet(7, rng)
    T, _, _, _ = O.solve_ugw(gx, gy, p, q, 1e9, 0.05, 3, 2000)
    Tb, _, _, _ = O.solve(gx, gy, p, q, 0.1, 3, 2000)
    assert np.max(np.abs(T - Tb)) <= 1e-6 * np.max(Tb)


@pytest.mark.parametrize("gx,gy", [(O.Grid((4,), 0.5, 1), O.Grid((3,), 0.5, 2)),
                                   (O.Grid((2, 2), 0.5, 1), O.Grid((3,), 0.25, 1))])
def test_objective_ugw_by_explicit_sums(gx, gy):
    rng = inputs.rng_for(945, gx.size, gy.size)
    M, N = gx.size, gy.size
    T = rng.uniform(0, 0.2, (M, N))
    u, v = rng.uniform(0.1, 0.5, M), rng.uniform(0.1, 0.5, N)
    rho, eps = 0.3, 0.02
    DX, DY = O.cost_matrix(gx), O.cost_matrix(gy)
    E = 0.0
    for i in range(M):
        for p in range(N):
            for j in range(M):
                for q in range(N):
                    E += (DX[i, j] - DY[p, q]) ** 2 * T[i, p] * T[j, q]
    a, b = T.sum(axis=1), T.sum(axis=0)
    U = E + rho * _kl_brute(np.outer(a, a), np.outer(u, u)) + rho * _kl_brute(np.outer(b, b), np.outer(v, v))
    uv = np.outer(u, v).ravel()
    R = U + eps * _kl_brute(np.outer(T.ravel(), T.ravel()), np.outer(uv, uv))
    got = O.objective_ugw(gx, gy, T, u, v, rho, eps)
    assert abs(got[0] - U) <= 1e-12 * abs(U) and abs(got[1] - R) <= 1e-12 * abs(R)


def test_ugw_shift_by_explicit_sums():
    rng = inputs.rng_for(946)
    T = rng.uniform(0, 0.3, (5, 4))
    T[1, 2] = 0.0
    u, v = rng.uniform(0.1, 1, 5), rng.uniform(0.1, 1, 4)
    rho, eps = 0.8, 0.03
    a, b = T.sum(axis=1), T.sum(axis=0)
    ref = rho * sum(x * math.log(x / y) for x, y in zip(a, u))
    ref += rho * sum(x * math.log(x / y) for x, y in zip(b, v))
    ref += eps * sum(T[i, p] * math.log(T[i, p] / (u[i] * v[p]))
                     for i in range(5) for p in range(4) if T[i, p] > 0)
    assert abs(O.ugw_shift(T, u, v, rho, eps) - ref) <= 1e-13 * abs(ref)
