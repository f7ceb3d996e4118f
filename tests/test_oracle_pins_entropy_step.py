"""More pins of the CPU oracle, each against a fact that does not come from the
oracle itself:

* the entropy H(T) = sum T (ln T - 1) of Sec. 2, Eq. (entropic GW), with
  0 ln 0 = 0: closed forms for the uniform coupling and for a product
  coupling p q^T (H = sum p ln p + sum q ln q - 1), and a hand-computed 2 x 2
  value; the second objective value is E + eps H;
* one mirror-descent step (Sec. 2.1, Eq. (GW sinkhorn) with the Remark on
  tau = eps): from T^0 = p q^T the plan is the Sinkhorn plan of the cost
  grad E(T^0), written here as the four-index sum of the gradient entry in
  exact rational arithmetic and solved by the scaling form u = p / (K v),
  v = q / (K^T u), K = exp(-C / eps);
* the unbalanced solve (Remark on UGW) on one-point grids, where D = 0 and the
  divergence reduces to a function of the single mass t whose minimiser is
  t* = (u v)^((rho + eps) / (2 rho + eps)).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import gw_oracle as O
from paper_2404_08970_amd import inputs


# ------------------------------------------------------------------ entropy

@pytest.mark.parametrize("M,N", [(1, 1), (3, 5), (16, 16), (7, 64)])
def test_entropy_uniform_coupling_closed_form(M, N):
    # T_ip = 1/(MN) everywhere: H = MN (1/(MN)) (ln(1/(MN)) - 1) = -ln(MN) - 1
    T = np.full((M, N), 1.0 / (M * N))
    assert abs(O.entropy(T) - (-math.log(M * N) - 1.0)) <= 1e-14 * (math.log(M * N) + 1.0)


def test_entropy_hand_computed_2x2_with_zero():
    # [[1/2, 1/4], [1/4, 0]]: 1/2 (-ln 2 - 1) + 2 (1/4)(-2 ln 2 - 1) + 0 = -3/2 ln 2 - 1
    T = np.array([[0.5, 0.25], [0.25, 0.0]])
    assert abs(O.entropy(T) - (-1.5 * math.log(2.0) - 1.0)) <= 1e-15


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_entropy_of_product_coupling(seed):
    # for normalised p, q: sum_ip p_i q_p (ln p_i + ln q_p - 1)
    #   = sum p ln p + sum q ln q - 1, with zero entries contributing nothing
    rng = inputs.rng_for(120, seed)
    p, q = inputs.dirichlet(40, rng), inputs.dirichlet(25, rng)
    p[[3, 17]] = 0.0
    q[[0, 24]] = 0.0
    p /= p.sum()
    q /= q.sum()
    ref = (math.fsum(x * math.log(x) for x in p if x > 0)
           + math.fsum(x * math.log(x) for x in q if x > 0) - 1.0)
    assert abs(O.entropy(np.outer(p, q)) - ref) <= 1e-13 * abs(ref)


def test_entropy_dyadic_entries_against_term_by_term_sum():
    # dyadic entries, several exactly zero; the reference sums x (ln x - 1) term by
    # term with a correctly rounded sum, skipping zeros (0 ln 0 = 0)
    rng = inputs.rng_for(121)
    T = rng.integers(0, 8, size=(9, 11)).astype(np.float64) / 64.0
    T[0, :] = 0.0
    ref = math.fsum(x * (math.log(x) - 1.0) for x in T.ravel() if x > 0)
    assert np.count_nonzero(T == 0) > 9
    assert abs(O.entropy(T) - ref) <= 1e-13 * abs(ref)


def test_objective_second_value_is_E_plus_eps_H():
    gx, gy = O.Grid((6,), 0.2, 2), O.Grid((5,), 0.25, 1)
    rng = inputs.rng_for(122)
    T = inputs.random_plan(6, 5, rng)
    T[2, 3] = 0.0
    # H from its definition for this T, summed term by term
    H = math.fsum(x * (math.log(x) - 1.0) for x in T.ravel() if x > 0)
    for eps in (0.0, 1e-3, 0.7):
        E, R = O.objective(gx, gy, T, eps)
        assert abs(R - (E + eps * H)) <= 1e-14 * (abs(E) + abs(eps * H))


# --------------------------------------------------- one mirror-descent step

def _four_index_gradient(DX, DY, T):
    """[grad E]_ip = 2 sum_j sum_q (dX_ij - dY_pq)^2 T_jq, exact rationals."""
    M, N = len(DX), len(DY)
    out = np.zeros((M, N))
    for i in range(M):
        for p in range(N):
            s = Fraction(0)
            for j in range(M):
                for q in range(N):
                    d = DX[i][j] - DY[p][q]
                    s += d * d * T[j][q]
            out[i, p] = float(2 * s)
    return out


def _scaling_form_plan(C, p, q, eps, iters):
    """u = p / (K v), v = q / (K^T u), plan = u_i K_ip v_p; v starts at 1."""
    M, N = C.shape
    K = [[math.exp(-C[i, j] / eps) for j in range(N)] for i in range(M)]
    v = [1.0] * N
    u = [1.0] * M
    for _ in range(iters):
        u = [p[i] / math.fsum(K[i][j] * v[j] for j in range(N)) for i in range(M)]
        v = [q[j] / math.fsum(K[i][j] * u[i] for i in range(M)) for j in range(N)]
    return np.array([[u[i] * K[i][j] * v[j] for j in range(N)] for i in range(M)])


@pytest.mark.parametrize("gx,gy,eps,inner", [
    (O.Grid((6,), 0.2, 1), O.Grid((5,), 0.25, 1), 0.05, 7),
    (O.Grid((5,), 0.25, 2), O.Grid((7,), 1 / 6, 3), 0.02, 12),
    (O.Grid((2, 3), 0.5, 2), O.Grid((4,), 1 / 3, 2), 0.1, 5),
    (O.Grid((3, 2), 0.5, 2, O.METRIC_SQEUCLID), O.Grid((2, 2), 0.5, 1), 0.05, 9),
])
def test_one_mirror_descent_step_is_scaling_sinkhorn_on_four_index_gradient(gx, gy, eps, inner):
    rng = inputs.rng_for(123, gx.size, gy.size)
    # dyadic marginals summing to 1 exactly, so p q^T has marginals p and q
    # exactly and the four-index sum is the gradient E's derivative at T^0
    a = rng.integers(1, 8, size=gx.size).astype(np.float64)
    b = rng.integers(1, 8, size=gy.size).astype(np.float64)
    p, q = a / a.sum(), b / b.sum()
    hx = Fraction(gx.h) ** (2 if gx.metric == O.METRIC_SQEUCLID else gx.k)
    hy = Fraction(gy.h) ** (2 if gy.metric == O.METRIC_SQEUCLID else gy.k)
    IX, IY = O.integer_distance(gx), O.integer_distance(gy)
    DX = [[hx * int(IX[i, j]) for j in range(gx.size)] for i in range(gx.size)]
    DY = [[hy * int(IY[i, j]) for j in range(gy.size)] for i in range(gy.size)]
    pf = [Fraction(int(x)) / int(a.sum()) for x in a]
    qf = [Fraction(int(x)) / int(b.sum()) for x in b]
    T0 = [[pf[i] * qf[j] for j in range(gy.size)] for i in range(gx.size)]
    C = _four_index_gradient(DX, DY, T0)
    ref = _scaling_form_plan(C, p, q, eps, inner)
    T1, _, _, _ = O.solve(gx, gy, p, q, eps, 1, inner)
    assert np.max(np.abs(T1 - ref)) <= 1e-12 * np.max(ref)
    T1p, _, _, _ = O.solve(gx, gy, p, q, eps, 1, inner, gradient="pascal")
    assert np.max(np.abs(T1p - ref)) <= 1e-12 * np.max(ref)


# ------------------------------------------------ UGW on one-point grids

@pytest.mark.parametrize("u,v,rho,eps", [(1.0, 1.5, 1.0, 0.2), (0.3, 2.0, 0.5, 0.1),
                                          (2.5, 0.7, 3.0, 1.0), (1e-3, 5.0, 0.2, 0.05),
                                          (4.0, 0.25, 1.0, 0.5)])
def test_solve_ugw_one_point_closed_form(u, v, rho, eps):
    """With one point per grid D = 0 and E = 0; with t the plan's mass, the
    divergence plus its entropic term is
      rho [t^2 ln(t^2/u^2) - t^2 + u^2] + rho [t^2 ln(t^2/v^2) - t^2 + v^2]
      + eps [t^2 ln(t^2/(uv)^2) - t^2 + (uv)^2],
    whose derivative 2t [(2 rho + eps) ln t^2 - (rho + eps) ln (uv)^2] vanishes at
    t* = (uv)^((rho + eps)/(2 rho + eps))."""
    g = O.Grid((1,), 1.0, 1)
    T, _, _, _ = O.solve_ugw(g, g, np.array([u]), np.array([v]), rho, eps, 10, 400)
    t_star = (u * v) ** ((rho + eps) / (2.0 * rho + eps))
    assert abs(T[0, 0] - t_star) <= 1e-14 * t_star
