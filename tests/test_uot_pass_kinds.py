"""The GPU parity cases of the unbalanced Sinkhorn exercise both kinds of
one-pass update (rows of up to 4096 entries; longer rows always run the
exact pass).

After the first pass of a call, a pass is shifted (each row shifted by the
previous pass's bound of its log-sum-exp plus D+, the column sums kept as
plain doubles in per-column frames) when D+ + D- <= 600, D+ <= 550 and the
band's row bounds stay below 1e6 - D+ in magnitude, D+ and D- being the
largest moves of g up and down (in units of e = eps here) over the columns
with v_p > 0 since the previous pass; otherwise it reduces the exact row
maxima.  The decision depends only on g and the row log-sum-exps, so it is
decided here from the oracle's potentials: the parity cases must contain
shifted passes, an exact pass after the first one, and a pass in which some
bands are exact and the others shifted."""
import numpy as np

from oracle import gw_oracle as O

from test_gpu_ugw import UOT_CASES, UOT_KINDS, uot_kinds_input
from paper_2404_08970_amd import inputs

SPREAD_MAX, UP_MAX, BOUND_MAX = 600.0, 550.0, 1.0e6


def _band_rows(M):
    rb = (M + 255) // 256
    return max((rb + 1) // 2 * 2, 2)


def _kinds(C, u, v, rho, eps, iters):
    """For passes 1..iters-1 of a cold-started call: the number of shifted
    bands and the number of bands."""
    M, N = C.shape
    inrow = v > 0
    lv = np.log(v[inrow])
    rb = _band_rows(M)
    nb = (M + rb - 1) // rb
    gs = [np.zeros(N)] + [O.uot_sinkhorn(C, u, v, rho, eps, t)[1] for t in range(1, iters)]
    out = []
    for t in range(1, iters):
        g, gp = gs[t][inrow], gs[t - 1][inrow]
        d = (g - gp) / eps
        up, dn = max(d.max(initial=0.0), 0.0), max((-d).max(initial=0.0), 0.0)
        # the row bounds of pass t - 1 (which used g before update t - 1)
        L = np.abs(O._lse_last_axis((gp[None, :] - C[:, inrow]) / eps + lv[None, :]))
        ok = up + dn <= SPREAD_MAX and up <= UP_MAX
        shifted = sum(ok and L[b * rb:(b + 1) * rb].max() + up < BOUND_MAX for b in range(nb))
        out.append((shifted, nb))
    return out


def test_uot_parity_cases_cover_both_pass_kinds():
    # a regular case: every pass after the first is shifted
    M, N, rho, eps, shift, iters = UOT_CASES[1]
    rng = inputs.rng_for(950, M, N)
    C = rng.uniform(0, 1, (M, N))
    u, v = rng.uniform(0.0, 2.0 / M, M), rng.uniform(0.0, 3.0 / N, N)
    u[M // 3] = 0.0
    v[[1, N // 2]] = 0.0
    assert all(s == nb for s, nb in _kinds(C + shift, u, v, rho, eps, iters))
    # sharp costs: the second pass falls back to the exact maxima, later ones are shifted
    M, N, rho, eps, scale, offset, iters = UOT_KINDS[0]
    k = _kinds(*uot_kinds_input(M, N, scale, offset), rho, eps, iters)
    assert k[0][0] == 0 and all(s == nb for s, nb in k[1:]), k
    # rows with a large cost offset: their band stays exact beside shifted ones
    M, N, rho, eps, scale, offset, iters = UOT_KINDS[1]
    k = _kinds(*uot_kinds_input(M, N, scale, offset), rho, eps, iters)
    assert all(0 < s < nb for s, nb in k), k
