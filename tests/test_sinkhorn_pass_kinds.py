"""The GPU Sinkhorn parity cases exercise both kinds of row pass.

A row pass after the first one of a call may run fast: shift each row by the
previous pass's upper bound of its log-sum-exp plus D+ (how far g moved up,
in units of eps) instead of reducing the row maximum, and keep the column sums
as plain doubles in fixed per-column frames, when D+ + D- <= 600, D+ <= 550
and the rows' bounds stay below 1e6 in magnitude; rows of more than 18
entries per thread (N > 9216) always take the exact maximum.  Whether a pass
is fast is a function of g before and after the previous column update (the
row bounds of these cases are far below the limit), so it can be decided here
from the oracle's potentials alone: the parity cases must contain fast passes
in every row-length class that allows them, and passes that fall back to the
exact maximum."""
import numpy as np

from oracle import gw_oracle as O
from paper_2404_08970_amd import inputs
from test_gpu_parity import SK_CASES

SPREAD_MAX = 600.0
UP_MAX = 550.0
BOUND_MAX = 1.0e6


def _moves(C, p, q, eps, iters):
    """(D+, D-, largest |row LSE|) seen by each row pass after the first
    (passes 1..iters-1 of a cold-started call): pass t compares g after update
    t with g before it (g = 0 before the first update); the row bounds are
    those of the previous pass, LSE_p((g_p - C_ip)/eps) with its g."""
    out = []
    g_prev = np.zeros(C.shape[1])
    for t in range(1, iters):
        _, g = O.sinkhorn(C, p, q, eps, t)
        bound = np.max(np.abs(O._lse_last_axis((g_prev[None, :] - C) / eps)))
        fin_n, fin_o = np.isfinite(g), np.isfinite(g_prev)
        if np.any(fin_n != fin_o):
            out.append((np.inf, np.inf, bound))
        else:
            d = (g[fin_n] - g_prev[fin_o]) / eps
            out.append((max(d.max(initial=0.0), 0.0), max((-d).max(initial=0.0), 0.0), bound))
        g_prev = g
    return out


def _fast(up, dn, bound):
    return up + dn <= SPREAD_MAX and up <= UP_MAX and bound + up < BOUND_MAX


def _spreads(C, p, q, eps, iters):
    return [u + d for u, d, _ in _moves(C, p, q, eps, iters)]


def test_parity_cases_cover_both_pass_kinds():
    shifted_classes, exact = set(), 0
    for M, N, eps, iters in SK_CASES:
        if iters < 2:
            continue
        rng = inputs.rng_for(205, M, N)
        C = rng.uniform(0, 2, size=(M, N))
        p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
        for up, dn, bound in _moves(2.0 * C, p, q, eps, iters):
            if _fast(up, dn, bound) and N <= 9216:
                shifted_classes.add(N)
            else:
                exact += 1
    # one fast case at least in each class that allows it (N <= 9216)
    bounds = [256, 512, 1024, 2048, 3072, 4096, 6144, 8192, 9216]
    covered = {next(b for b in bounds if n <= b) for n in shifted_classes}
    assert covered == set(bounds), sorted(covered)
    assert exact > 0


def test_spread_of_the_first_update_exceeds_the_limit_on_peaked_costs():
    """With C/eps in the thousands the first update moves g by far more than
    600 eps, so the second pass takes the exact maxima; later passes move g by
    little and are shifted (the GPU parity tests run this cost with positive
    marginals and with zero-mass rows and columns)."""
    rng = inputs.rng_for(206)
    M, N = 90, 70
    C = rng.uniform(0, 4, size=(M, N))
    C[:, 5] += 3.0
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    s = _spreads(C, p, q, 1e-3, 4)
    assert s[0] > SPREAD_MAX and s[1] <= SPREAD_MAX and s[2] <= SPREAD_MAX
    # a zero-mass column turns -inf in the first update: the move is unbounded
    q[[3, 69]] = 0.0; q /= q.sum()
    assert _spreads(C, p, q, 1e-3, 2)[0] == np.inf
