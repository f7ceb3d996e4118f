"""Pins of the oracle's tolerance-stopped Sinkhorn against facts that do not
come from its own log-domain arithmetic: the closed form of Sinkhorn on a
separable cost (exact after one full iteration), and the marginal-violation
trajectory of the scaling form u = p / (K v), v = q / (K^T u)."""
import numpy as np
import pytest

from oracle import gw_oracle as O
from paper_2404_08970_amd import inputs


def _scaling_errors(C, p, q, eps, iters):
    """err_t = || v_{t-1} o (K^T u_t) - q ||_1 for t = 1..iters (scaling form,
    cold start v_0 = 1): the column sums of the plan after the row scaling."""
    K = np.exp(-C / eps)
    v = np.ones(C.shape[1])
    errs = []
    for _ in range(iters):
        u = p / (K @ v)
        col = v * (K.T @ u)
        errs.append(float(np.sum(np.abs(col - q))))
        with np.errstate(divide="ignore", invalid="ignore"):
            v = np.where(q > 0, q / (K.T @ u), 0.0)
    return errs


def test_separable_cost_closed_form():
    """C_ip = a_i + b_p: K = u v^T has rank one, so after the first row update
    the plan is p_i v_p / sum(v) and its column violation is
    sum_p |v_p / sum(v) - q_p|; the first g update makes both marginals exact,
    so with check_every = 1 and a small tol the loop stops at t = 2."""
    rng = inputs.rng_for(900)
    M, N, eps = 9, 7, 0.3
    a, b = rng.uniform(0, 1, M), rng.uniform(0, 1, N)
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    C = a[:, None] + b[None, :]
    v = np.exp(-b / eps)
    err1 = float(np.sum(np.abs(v / v.sum() - q)))
    assert err1 > 1e-3
    f, g, k, err = O.sinkhorn_tol(C, p, q, eps, 50, 1, 1e-12)
    assert k == 2 and err <= 1e-13
    f1, g1, k1, e1 = O.sinkhorn_tol(C, p, q, eps, 50, 1, 1.001 * err1)
    assert k1 == 1 and abs(e1 - err1) <= 1e-14
    P = O.plan(C, f1, g1, eps)
    assert np.max(np.abs(P.sum(axis=0) - q)) <= 1e-15
    assert np.max(np.abs(P.sum(axis=1) - p)) <= 1e-14


@pytest.mark.parametrize("M,N,eps,every,zeros", [(12, 10, 0.05, 1, False), (15, 11, 0.02, 3, False),
                                                  (10, 13, 0.04, 2, True)])
def test_stop_matches_scaling_form_trajectory(M, N, eps, every, zeros):
    rng = inputs.rng_for(901, M, N, every)
    C = rng.uniform(0, 1, size=(M, N))
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    if zeros:
        p[3] = 0.0
        q[[0, 5]] = 0.0
        p, q = p / p.sum(), q / q.sum()
    iters = 60
    errs = _scaling_errors(C, p, q, eps, iters)
    checked = [t for t in range(1, iters + 1) if t % every == 0]
    # tol between two consecutive checked errors, away from both
    for j in (2, 5, 9):
        hi, lo = errs[checked[j - 1] - 1], errs[checked[j] - 1]
        assert lo < 0.9 * hi  # a clear gap: the rounding of err cannot decide
        tol = (hi * lo) ** 0.5
        first = next(t for t in checked if errs[t - 1] <= tol)
        f, g, k, err = O.sinkhorn_tol(C, p, q, eps, iters, every, tol)
        assert k == first
        assert abs(err - errs[k - 1]) <= 1e-12 * max(errs[k - 1], 1e-300) + 1e-15
        f2, g2 = O.sinkhorn(C, p, q, eps, k)
        assert np.array_equal(f, f2) and np.array_equal(g, g2)


def test_never_checked_is_plain_sinkhorn():
    rng = inputs.rng_for(902)
    C = rng.uniform(0, 1, size=(8, 6))
    p, q = inputs.dirichlet(8, rng), inputs.dirichlet(6, rng)
    f, g, k, err = O.sinkhorn_tol(C, p, q, 0.1, 7, 10, 1.0)
    f2, g2 = O.sinkhorn(C, p, q, 0.1, 7)
    assert k == 7 and np.isnan(err)
    assert np.array_equal(f, f2) and np.array_equal(g, g2)


def test_solve_tol_counts():
    gx, gy = O.Grid((20,), 1 / 19, 1), O.Grid((16,), 1 / 15, 2)
    rng = inputs.rng_for(903)
    p, q = inputs.gauss_mixture_1d(20, rng), inputs.gauss_mixture_1d(16, rng)
    T, f, g, obj, done = O.solve_tol(gx, gy, p, q, 0.05, 3, 200, 5, 1e-9)
    assert len(done) == 3 and all(k % 5 == 0 and k <= 200 for k in done)
    _, _, _, _, d1 = O.solve_tol(gx, gy, p, q, 0.05, 1, 200, 5, 1e-9)
    assert d1 == done[:1]
    # the stopped plan meets the tolerance on the rows and exactly on the columns
    assert np.sum(np.abs(T.sum(axis=0) - q)) <= 1e-12
