"""Pins of the CPU oracle against facts that do not come from the oracle itself:
the paper's printed matrices, brute-force four-index sums in exact rational
arithmetic, closed forms of the recursion, exact integer arithmetic, invariances
of the GW objective and textbook properties of Sinkhorn's iteration."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import gw_oracle as O
from paper_2404_08970_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_blocks(name):
    blocks, cur = [], []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line:
                continue
            if line.startswith("#"):
                if cur:
                    blocks.append(np.array(cur, dtype=np.float64))
                    cur = []
                continue
            cur.append([float(t) for t in line.split()])
    if cur:
        blocks.append(np.array(cur, dtype=np.float64))
    return blocks


# ---------------------------------------------------------------- grid indexing

@pytest.mark.parametrize("k", [1, 2, 3])
def test_1d_distance_is_paper_L_plus_LT(k):
    (L1,) = _read_blocks("paper_L_n5.txt")
    L = L1 ** k
    D = O.integer_distance(O.Grid((5,), 1.0, k)).astype(np.float64)
    assert np.array_equal(D, L + L.T)


def test_D1_and_J_fixture_match_grid():
    D1, J = _read_blocks("paper_D1_J_n4.txt")
    assert np.array_equal(O.integer_distance(O.Grid((4,), 1.0, 1)), D1)
    assert np.array_equal(O.toeplitz_apply(np.eye(4), 0), J)


def test_2d_distance_matches_printed_block_form_n2():
    Dk1, Dk2 = _read_blocks("paper_Dhat_n2.txt")
    assert np.array_equal(O.integer_distance(O.Grid((2, 2), 1.0, 1)), Dk1)
    assert np.array_equal(O.integer_distance(O.Grid((2, 2), 1.0, 2)), Dk2)


@pytest.mark.parametrize("n,k", [(3, 1), (3, 2), (4, 3), (5, 2)])
def test_2d_distance_matches_block_formula(n, k):
    # block (a, a') of D^ is (D_1 + |a - a'| J)^{ok}, Sec. 3.1 Eq. (2d Dx)
    D1 = np.abs(np.subtract.outer(np.arange(n), np.arange(n)))
    Dhat = np.block([[(D1 + abs(a - b)) ** k for b in range(n)] for a in range(n)])
    assert np.array_equal(O.integer_distance(O.Grid((n, n), 1.0, k)), Dhat)


def test_2d_kronecker_expansion_identity():
    # D^ = sum_r C(k,r) D_1^{or} (x) D_1^{o(k-r)} with D_1^{o0} = J (Sec. 3.1)
    n = 4
    D1 = np.abs(np.subtract.outer(np.arange(n), np.arange(n))).astype(np.int64)
    for k in (1, 2, 3):
        S = sum(math.comb(k, r) * np.kron(D1 ** r, D1 ** (k - r)) for r in range(k + 1))
        assert np.array_equal(S, O.integer_distance(O.Grid((n, n), 1.0, k)))


def test_sqeuclid_distance_from_coordinates():
    H, W = 3, 4
    D = O.integer_distance(O.Grid((H, W), 1.0, 2, O.METRIC_SQEUCLID))
    for i in range(H * W):
        for j in range(H * W):
            r, c, r2, c2 = i // W, i % W, j // W, j % W
            assert D[i, j] == (r - r2) ** 2 + (c - c2) ** 2


# ---------------------------------------------------- gradient vs four-index sum

def _frac_grid_matrix(g):
    hk = Fraction(g.h) ** (2 if g.metric == O.METRIC_SQEUCLID else g.k)
    Di = O.integer_distance(g)
    return [[hk * int(Di[i, j]) for j in range(Di.shape[1])] for i in range(Di.shape[0])]


def _four_index_half_gradient(gx, gy, T):
    """[grad E]_ip / 2 = sum_j sum_q (dX_ij - dY_pq)^2 T_jq (Eq. gradient entry),
    in exact rational arithmetic."""
    DX, DY = _frac_grid_matrix(gx), _frac_grid_matrix(gy)
    M, N = len(DX), len(DY)
    Tf = [[Fraction(float(T[j, q])) for q in range(N)] for j in range(M)]
    out = np.zeros((M, N))
    for i in range(M):
        for p in range(N):
            s = Fraction(0)
            for j in range(M):
                for q in range(N):
                    d = DX[i][j] - DY[p][q]
                    s += d * d * Tf[j][q]
            out[i, p] = float(s)
    return out


CASES = [
    (O.Grid((5,), 0.25, 1), O.Grid((5,), 0.25, 1)),
    (O.Grid((6,), 0.25, 2), O.Grid((4,), 0.5, 3)),
    (O.Grid((2, 3), 0.5, 1), O.Grid((3, 2), 0.25, 2)),
    (O.Grid((2, 2), 0.5, 2, O.METRIC_SQEUCLID), O.Grid((5,), 0.25, 2)),
]


@pytest.mark.parametrize("gx,gy", CASES)
def test_grad_dense_equals_four_index_sum(gx, gy):
    rng = inputs.rng_for(101, gx.size, gy.size)
    T = rng.integers(0, 64, size=(gx.size, gy.size)) / 64.0
    p, q = T.sum(axis=1), T.sum(axis=0)       # the identity needs T's own marginals
    ref = _four_index_half_gradient(gx, gy, T)
    G = O.grad_dense(gx, gy, p, q, T)
    assert np.max(np.abs(G - ref)) <= 1e-14 * np.max(np.abs(ref))
    Gp = O.grad_pascal(gx, gy, p, q, T)
    assert np.max(np.abs(Gp - ref)) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("gx,gy", CASES)
def test_objective_equals_four_index_qap(gx, gy):
    rng = inputs.rng_for(102, gx.size, gy.size)
    T = rng.integers(0, 16, size=(gx.size, gy.size)) / 64.0
    DX, DY = _frac_grid_matrix(gx), _frac_grid_matrix(gy)
    M, N = T.shape
    Tf = [[Fraction(float(T[i, p])) for p in range(N)] for i in range(M)]
    E = Fraction(0)
    for i in range(M):
        for j in range(M):
            for p in range(N):
                if Tf[i][p] == 0:
                    continue
                for q in range(N):
                    d = DX[i][j] - DY[p][q]
                    E += d * d * Tf[i][p] * Tf[j][q]
    got, _ = O.objective(gx, gy, T, 0.01)
    assert abs(got - float(E)) <= 1e-14 * abs(float(E))


# ------------------------------------------------------- recursion, exactly

@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_lower_apply_closed_form_integers(m):
    rng = inputs.rng_for(103, m)
    n = 200
    x = rng.integers(0, 1000, size=n)
    y = O.lower_apply(x.astype(np.float64), m)
    # y_i = sum_r C(m,r) i^{m-r} (-1)^r S_r(i), S_r(i) = sum_{j<i} j^r x_j, in Python ints
    for i in range(n):
        exact = 0
        for r in range(m + 1):
            S = sum(int(j) ** r * int(x[j]) for j in range(i))
            exact += math.comb(m, r) * i ** (m - r) * (-1) ** r * S
        assert y[i] == float(exact)


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_toeplitz_apply_matches_explicit_matrix_exactly(m):
    rng = inputs.rng_for(104, m)
    n = 37
    X = rng.integers(0, 50, size=(n, 3)).astype(np.float64)
    idx = np.arange(n)
    Dm = np.abs(idx[:, None] - idx[None, :]).astype(np.int64) ** m
    exact = Dm @ X.astype(np.int64)
    assert np.array_equal(O.toeplitz_apply(X, m), exact.astype(np.float64))


def test_upper_is_transpose_of_lower():
    rng = inputs.rng_for(105)
    n = 30
    x = rng.integers(0, 20, size=(n, 2)).astype(np.float64)
    idx = np.arange(n)
    for m in (1, 2, 3):
        L = np.where(idx[:, None] > idx[None, :], (idx[:, None] - idx[None, :]) ** m, 0)
        assert np.array_equal(O.lower_apply(x, m), (L @ x.astype(np.int64)).astype(float))
        assert np.array_equal(O.upper_apply(x, m), (L.T @ x.astype(np.int64)).astype(float))


@pytest.mark.parametrize("g", [O.Grid((3, 4), 1.0, 1), O.Grid((4, 3), 1.0, 2),
                               O.Grid((3, 3), 1.0, 3),
                               O.Grid((4, 5), 1.0, 2, O.METRIC_SQEUCLID)])
def test_grid_apply_matches_explicit_matrix_exactly(g):
    rng = inputs.rng_for(106, g.size, g.k)
    X = rng.integers(0, 30, size=(g.size, 4)).astype(np.float64)
    exact = O.integer_distance(g) @ X.astype(np.int64)
    assert np.array_equal(O.grid_apply(g, X), exact.astype(np.float64))


@pytest.mark.parametrize("gx,gy", [
    (O.Grid((40,), 1.0, 1), O.Grid((33,), 1.0, 2)),
    (O.Grid((25,), 1.0, 3), O.Grid((25,), 1.0, 3)),
    (O.Grid((4, 5), 1.0, 2), O.Grid((3, 3), 1.0, 1)),
    (O.Grid((5, 4), 1.0, 2, O.METRIC_SQEUCLID), O.Grid((4, 4), 1.0, 2, O.METRIC_SQEUCLID)),
])
def test_grad_pascal_bit_exact_on_integer_inputs(gx, gy):
    rng = inputs.rng_for(107, gx.size, gy.size)
    T = inputs.integer_plan(gx.size, gy.size, rng)
    p = rng.integers(0, 5, size=gx.size).astype(np.float64)
    q = rng.integers(0, 5, size=gy.size).astype(np.float64)
    assert np.array_equal(O.grad_pascal(gx, gy, p, q, T), O.grad_dense(gx, gy, p, q, T))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_grad_pascal_close_to_dense_on_plans(k):
    rng = inputs.rng_for(108, k)
    n = 300
    g = O.Grid((n,), 1.0 / (n - 1), k)
    T = inputs.peaked_plan(n, n, rng)
    p, q = inputs.dirichlet(n, rng), inputs.dirichlet(n, rng)
    Gd = O.grad_dense(g, g, p, q, T)
    Gp = O.grad_pascal(g, g, p, q, T)
    assert np.max(np.abs(Gd - Gp)) <= 1e-13 * np.max(np.abs(Gd))


@pytest.mark.parametrize("g", [O.Grid((9,), 1.0, 2), O.Grid((3, 4), 1.0, 2),
                               O.Grid((3, 3), 1.0, 2, O.METRIC_SQEUCLID)])
def test_impulse_gradient_exact(g):
    # T = e_j e_q^T, p = e_j, q = e_q, h = 1  =>  G_ip = (D_ij - D_qp)^2
    D = O.integer_distance(g).astype(np.float64)
    n = g.size
    for j, q_ in [(0, n - 1), (n // 2, 1), (2, 2)]:
        T = np.zeros((n, n)); T[j, q_] = 1.0
        p = np.zeros(n); p[j] = 1.0
        q = np.zeros(n); q[q_] = 1.0
        ref = (D[:, j][:, None] - D[q_, :][None, :]) ** 2
        assert np.array_equal(O.grad_dense(g, g, p, q, T), ref)
        assert np.array_equal(O.grad_pascal(g, g, p, q, T), ref)


def test_gradient_reflection_equivariance():
    rng = inputs.rng_for(109)
    n = 50
    g = O.Grid((n,), 1.0 / (n - 1), 2)
    T = inputs.random_plan(n, n, rng)
    p, q = T.sum(1), T.sum(0)
    G = O.grad_pascal(g, g, p, q, T)
    Gr = O.grad_pascal(g, g, p[::-1], q, T[::-1])
    assert np.max(np.abs(Gr - G[::-1])) <= 1e-14 * np.max(np.abs(G))


# ------------------------------------------------------------------- objective

def test_objective_zero_at_identity_coupling():
    n = 64                                  # dyadic uniform mass, h = 1
    g = O.Grid((n,), 1.0, 2)
    T = np.eye(n) / n
    E, _ = O.objective(g, g, T, 0.0)
    assert E == 0.0
    g2 = O.Grid((8, 8), 1.0, 1)
    E2, _ = O.objective(g2, g2, np.eye(64) / 64, 0.0)
    assert E2 == 0.0


def test_objective_nonnegative_and_reflection_invariant():
    rng = inputs.rng_for(110)
    n = 40
    gx = O.Grid((n,), 1.0 / (n - 1), 1)
    gy = O.Grid((n,), 1.0 / (n - 1), 2)
    for _ in range(3):
        T = inputs.random_plan(n, n, rng)
        E, _ = O.objective(gx, gy, T, 0.0)
        Er, _ = O.objective(gx, gy, T[::-1, ::-1], 0.0)
        assert E >= 0
        assert abs(E - Er) <= 1e-13 * abs(E)


# -------------------------------------------------------------------- Sinkhorn

def _scaling_sinkhorn(C, p, q, eps, iters):
    """The same iteration in the scaling form u = p/(K v), v = q/(K^T u)."""
    K = np.exp(-C / eps)
    v = np.ones(C.shape[1])
    for _ in range(iters):
        u = p / (K @ v)
        v = q / (K.T @ u)
    return eps * np.log(u), eps * np.log(v)


def test_sinkhorn_matches_scaling_form():
    rng = inputs.rng_for(111)
    M, N = 37, 29
    C = rng.uniform(0, 1, size=(M, N))
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    eps = 0.05
    f, g = O.sinkhorn(C, p, q, eps, 50)
    fs, gs = _scaling_sinkhorn(C, p, q, eps, 50)
    assert np.max(np.abs(f - fs)) <= 1e-12
    assert np.max(np.abs(g - gs)) <= 1e-12


def test_sinkhorn_constant_cost_gives_product_plan():
    rng = inputs.rng_for(112)
    M, N = 20, 30
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    C = np.full((M, N), 0.7)
    f, g = O.sinkhorn(C, p, q, 0.01, 1)
    P = O.plan(C, f, g, 0.01)
    assert np.max(np.abs(P - np.outer(p, q))) <= 1e-15


def test_sinkhorn_marginals():
    rng = inputs.rng_for(113)
    M, N = 60, 50
    C = rng.uniform(0, 1, size=(M, N))
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    eps = 0.02
    errs = []
    for it in (1, 10, 100, 2000):
        f, g = O.sinkhorn(C, p, q, eps, it)
        P = O.plan(C, f, g, eps)
        assert np.max(np.abs(P.sum(0) - q)) <= 1e-15     # column marginal after g update
        errs.append(np.max(np.abs(P.sum(1) - p)))
    assert errs[-1] <= 1e-12
    assert errs[-1] < errs[1] < errs[0]


def test_sinkhorn_dual_monotone():
    rng = inputs.rng_for(114)
    M, N = 30, 40
    C = rng.uniform(0, 1, size=(M, N))
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    eps = 0.05
    prev = -np.inf
    f = g = None
    for _ in range(30):
        f, g = O.sinkhorn(C, p, q, eps, 1, f, g)
        dual = f @ p + g @ q - eps * np.sum(O.plan(C, f, g, eps))
        assert dual >= prev - 1e-15
        prev = dual


def test_sinkhorn_zero_mass_entries():
    rng = inputs.rng_for(115)
    M, N = 12, 9
    C = rng.uniform(0, 1, size=(M, N))
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    p[3] = 0.0; p /= p.sum()
    q[0] = 0.0; q[5] = 0.0; q /= q.sum()
    f, g = O.sinkhorn(C, p, q, 0.05, 200)
    assert np.isneginf(f[3]) and np.isneginf(g[0]) and np.isneginf(g[5])
    P = O.plan(C, f, g, 0.05)
    assert np.all(np.isfinite(P))
    assert np.all(P[3] == 0) and np.all(P[:, 0] == 0)
    assert np.max(np.abs(P.sum(0) - q)) <= 1e-15


def test_sinkhorn_large_cost_over_eps_stays_finite():
    # C/eps up to 4000: the scaling form underflows, the log form must not
    rng = inputs.rng_for(116)
    M, N = 50, 40
    C = rng.uniform(0, 4, size=(M, N))
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    f, g = O.sinkhorn(C, p, q, 1e-3, 20)
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(g))
    P = O.plan(C, f, g, 1e-3)
    # exponents reach C/eps = 4000, so each plan entry carries ~4000 ulp of rounding
    assert np.max(np.abs(P.sum(0) - q) / q) <= 1e-12


# ----------------------------------------------------------------------- solve

def test_solve_fast_vs_dense_plan_agreement_table2():
    # Table 2's fast-vs-original plan gap is ~5e-15 at N = 500 (k = 1, eps = 0.002,
    # 10 outer iterations); the two oracle gradients must agree to that order.
    rows = _read_blocks("paper_table2_gw.txt")[0]
    N = int(rows[0, 0]); paper_gap = rows[0, 4]
    rng = inputs.rng_for(117, N)
    p, q = inputs.uniform_marginal(N, rng), inputs.uniform_marginal(N, rng)
    g = O.Grid((N,), 1.0 / (N - 1), 1)
    Td, *_ = O.solve(g, g, p, q, 0.002, 10, 30, gradient="dense")
    Tf, *_ = O.solve(g, g, p, q, 0.002, 10, 30, gradient="pascal")
    gap = np.linalg.norm(Td - Tf)
    assert gap <= 20 * paper_gap


def test_solve_small_properties():
    rng = inputs.rng_for(118)
    n = 40
    g = O.Grid((n,), 1.0 / (n - 1), 2)
    p, q = inputs.gauss_mixture_1d(n, rng), inputs.gauss_mixture_1d(n, rng)
    T, f, gg, (E, Ereg) = O.solve(g, g, p, q, 5e-3, 5, 50)
    assert np.max(np.abs(T.sum(0) - q)) <= 1e-15
    assert E >= 0
    T0 = np.outer(p, q)
    E0, _ = O.objective(g, g, T0, 5e-3)
    assert E < E0


# ------------------------------------------------------------ sampled rows

@pytest.mark.parametrize("gx,gy", [
    (O.Grid((37,), 1 / 36, 2), O.Grid((41,), 1 / 40, 3)),
    (O.Grid((5, 7), 1 / 6, 1), O.Grid((6, 4), 1 / 5, 2)),
    (O.Grid((6, 6), 1 / 5, 2, O.METRIC_SQEUCLID), O.Grid((30,), 1 / 29, 2)),
])
def test_grad_rows_equals_grad_dense(gx, gy):
    """The blocked row evaluation used at full sizes is the plain definition:
    it reproduces every row of grad_dense (block sizes that split D_Y)."""
    rng = np.random.default_rng([17, gx.size, gy.size])
    p = rng.dirichlet(np.ones(gx.size))
    q = rng.dirichlet(np.ones(gy.size))
    T = rng.uniform(0, 1, size=(gx.size, gy.size))
    G = O.grad_dense(gx, gy, p, q, T)
    rows = np.arange(gx.size)
    for block in (1, 7, 1024):
        Gr = O.grad_rows(gx, gy, p, q, T, rows, block=block)
        assert np.max(np.abs(Gr - G)) <= 1e-13 * np.max(np.abs(G))


def test_grad_rows_integer_inputs_exact():
    """Integer plan, unit spacing and integer marginals: every value is an
    integer below 2^53, so the sampled rows equal the full matrix exactly."""
    g = O.Grid((50,), 1.0, 2)
    rng = np.random.default_rng(18)
    T = rng.integers(0, 5, size=(50, 50)).astype(float)
    p = rng.integers(0, 3, size=50).astype(float)
    q = rng.integers(0, 3, size=50).astype(float)
    G = O.grad_dense(g, g, p, q, T)
    rows = np.array([0, 17, 49])
    assert np.array_equal(O.grad_rows(g, g, p, q, T, rows, block=16), G[rows])


def test_integer_distance_rows_match():
    for g in (O.Grid((9,), 1.0, 3), O.Grid((4, 5), 1.0, 2), O.Grid((3, 6), 1.0, 2, O.METRIC_SQEUCLID)):
        D = O.integer_distance(g)
        rows = np.arange(g.size)[::2]
        assert np.array_equal(O.integer_distance_rows(g, rows), D[rows])
