"""GPU parity of unbalanced GW (Remark on UGW) against the oracle: the
unbalanced Sinkhorn in every row-length class (zero-mass entries, a cost
shift, warm start; one row, one column, costs up to 1000 eps) and the UGW solve on 1D (FAST and dense), 2D and mixed grids,
including outer = 0 and the n = 1024 problem in full."""
import math

import numpy as np
import pytest

from oracle import gw_oracle as O
from paper_2404_08970_amd import inputs

from test_gpu_parity import TOL, _gw, _to_dev, err, ogrid

pytestmark = pytest.mark.gpu


UOT_CASES = [(37, 100, 0.5, 0.05, 0.0, 5), (64, 700, 2.0, 0.02, 0.3, 8), (20, 1500, 0.1, 0.03, -0.2, 6),
             (40, 3000, 1.0, 0.05, 0.0, 4), (33, 4096, 0.3, 0.01, 0.1, 5), (17, 5000, 5.0, 0.05, 0.0, 3),
             (12, 9000, 0.7, 0.02, 0.05, 4), (9, 16384, 1.5, 0.05, 0.0, 3)]


@pytest.mark.parametrize("M,N,rho,eps,shift,iters", UOT_CASES)
def test_uot_sinkhorn_matches_oracle(M, N, rho, eps, shift, iters):
    gw, torch = _gw()
    print(f"uot M={M} N={N} rho={rho} eps={eps}", flush=True)
    rng = inputs.rng_for(950, M, N)
    C = rng.uniform(0, 1, (M, N))
    u, v = rng.uniform(0.0, 2.0 / M, M), rng.uniform(0.0, 3.0 / N, N)
    u[M // 3] = 0.0
    v[[1, N // 2]] = 0.0
    f0, g0 = O.uot_sinkhorn(C + shift, u, v, rho, eps, iters)
    T0 = O.uot_plan(C + shift, f0, g0, u, v, eps)
    d = lambda a: _to_dev(torch, a)
    f, g, T = gw.uot_sinkhorn(d(C), d(u), d(v), rho, eps, iters, c_shift=shift, plan=True)
    torch.cuda.synchronize()
    assert err(f.cpu().numpy(), f0) <= TOL
    assert err(g.cpu().numpy(), g0) <= TOL
    assert err(T.cpu().numpy(), T0) <= TOL


UOT_EDGE = [(700, 300, 1.0, 0.002, 0.0, 4),    # 175 bands of 4 rows, C/eps up to 500
            (1, 5000, 0.5, 0.01, 0.0, 3),      # one row
            (3000, 1, 0.5, 0.01, 0.0, 3),      # one column
            (513, 2048, 2.0, 0.001, 0.0, 3)]   # C/eps up to 1000, a ragged last band


@pytest.mark.parametrize("M,N,rho,eps,shift,iters", UOT_EDGE)
def test_uot_sinkhorn_edge_shapes_match_oracle(M, N, rho, eps, shift, iters):
    """Shapes at the edges of the one-pass update's banding, and costs far
    above eps, where a column's largest term lies many binades below the row
    maxima of the pass (the extended-exponent column sums)."""
    gw, torch = _gw()
    print(f"uot edge M={M} N={N} rho={rho} eps={eps}", flush=True)
    rng = inputs.rng_for(951, M, N)
    C = rng.uniform(0, 1, (M, N))
    u, v = rng.uniform(0.0, 2.0 / M, M), rng.uniform(0.0, 3.0 / N, N)
    if M > 2:
        u[M // 3] = 0.0
    if N > 2:
        v[[1, N // 2]] = 0.0
    f0, g0 = O.uot_sinkhorn(C + shift, u, v, rho, eps, iters)
    T0 = O.uot_plan(C + shift, f0, g0, u, v, eps)
    d = lambda a: _to_dev(torch, a)
    f, g, T = gw.uot_sinkhorn(d(C), d(u), d(v), rho, eps, iters, c_shift=shift, plan=True)
    torch.cuda.synchronize()
    assert err(f.cpu().numpy(), f0) <= TOL
    assert err(g.cpu().numpy(), g0) <= TOL
    assert err(T.cpu().numpy(), T0) <= TOL


# The one-pass update runs its first pass of a call exact and later passes
# shifted (row shift from the previous bound, column sums in per-column
# frames) when the moves of g allow.  Two cases for the other combinations:
# costs up to 30000 e, whose first update moves g by more than 600 e, so the
# second pass falls back to exact maxima; and three rows with a cost offset of
# 1.2e4 (row bounds near -1.2e6), whose band stays exact beside shifted bands.
# tests/test_uot_pass_kinds.py checks both from the oracle's potentials.
UOT_KINDS = [(150, 1100, 20.0, 0.0002, 6.0, 0.0, 4), (600, 700, 0.5, 0.01, 1.0, 1.2e4, 4)]


def uot_kinds_input(M, N, scale, offset):
    rng = inputs.rng_for(952, M, N)
    C = rng.uniform(0, scale, (M, N))
    if offset:
        C[M // 2: M // 2 + 3] += offset
    u, v = rng.uniform(0.0, 2.0 / M, M), rng.uniform(0.0, 3.0 / N, N)
    u[M // 3] = 0.0
    v[[1, N // 2]] = 0.0
    return C, u, v


@pytest.mark.parametrize("M,N,rho,eps,scale,offset,iters", UOT_KINDS)
def test_uot_sinkhorn_pass_kinds_match_oracle(M, N, rho, eps, scale, offset, iters):
    gw, torch = _gw()
    print(f"uot kinds M={M} N={N} rho={rho} eps={eps} offset={offset}", flush=True)
    C, u, v = uot_kinds_input(M, N, scale, offset)
    f0, g0 = O.uot_sinkhorn(C, u, v, rho, eps, iters)
    T0 = O.uot_plan(C, f0, g0, u, v, eps)
    d = lambda a: _to_dev(torch, a)
    f, g, T = gw.uot_sinkhorn(d(C), d(u), d(v), rho, eps, iters, plan=True)
    torch.cuda.synchronize()
    assert err(f.cpu().numpy(), f0) <= TOL
    assert err(g.cpu().numpy(), g0) <= TOL
    assert err(T.cpu().numpy(), T0) <= TOL


def test_uot_warm_start():
    gw, torch = _gw()
    rng = inputs.rng_for(951)
    C = rng.uniform(0, 1, (50, 300))
    u, v = rng.uniform(0.01, 0.03, 50), rng.uniform(0.001, 0.005, 300)
    fw, gw0 = O.uot_sinkhorn(C, u, v, 0.8, 0.04, 3)
    f0, g0 = O.uot_sinkhorn(C, u, v, 0.8, 0.04, 5, fw, gw0)
    d = lambda a: _to_dev(torch, a)
    f, g = gw.uot_sinkhorn(d(C), d(u), d(v), 0.8, 0.04, 5, f=d(fw), g=d(gw0))
    torch.cuda.synchronize()
    assert err(f.cpu().numpy(), f0) <= TOL and err(g.cpu().numpy(), g0) <= TOL


SOLVE_CASES = [((80,), 1, 0, (64,), 2, 0, 1.0, 0.02, 3, 30, "fast"),
               ((120,), 2, 0, (100,), 1, 0, 0.2, 0.05, 2, 40, "dense"),
               ((9, 10), 1, 0, (11, 8), 2, 1, 3.0, 0.03, 3, 25, "fast"),
               ((4, 4, 5), 1, 0, (70,), 1, 0, 0.5, 0.02, 2, 30, "fast")]


def _measures(X, rng, mass):
    if X.ndim == 1:
        w = inputs.gauss_mixture_1d(X.size, rng)
    elif X.ndim == 2:
        w = inputs.blobs_2d(X.shape[0], X.shape[1], rng, floor=1e-6)
    else:
        w = inputs.blobs_3d(*X.shape, rng, floor=1e-6)
    return mass * w


@pytest.mark.parametrize("sx,kx,mx,sy,ky,my,rho,eps,outer,inner,path", SOLVE_CASES)
def test_solve_ugw_matches_oracle(sx, kx, mx, sy, ky, my, rho, eps, outer, inner, path):
    gw, torch = _gw()
    print(f"ugw {sx} {sy} rho={rho} eps={eps} {outer}x{inner} {path}", flush=True)
    X, Y = gw.unit_grid(sx, kx, mx), gw.unit_grid(sy, ky, my)
    rng = inputs.rng_for(952, X.size, Y.size)
    u, v = _measures(X, rng, 1.0), _measures(Y, rng, 1.6)
    T0, f0, g0, (U0, R0) = O.solve_ugw(ogrid(X), ogrid(Y), u, v, rho, eps, outer, inner)
    T, f, g, obj = gw.solve_ugw(X, Y, _to_dev(torch, u), _to_dev(torch, v), rho, eps, outer,
                                inner, path=path)
    torch.cuda.synchronize()
    assert err(T.cpu().numpy(), T0) <= TOL
    assert err(f.cpu().numpy(), f0) <= TOL and err(g.cpu().numpy(), g0) <= TOL
    o = obj.cpu().numpy()
    assert abs(o[0] - U0) <= TOL * abs(U0) and abs(o[1] - R0) <= TOL * abs(R0)


def test_solve_ugw_zero_steps():
    gw, torch = _gw()
    X, Y = gw.unit_grid((30,), 1), gw.unit_grid((25,), 2)
    rng = inputs.rng_for(953)
    u, v = rng.uniform(0, 0.1, 30), rng.uniform(0, 0.2, 25)
    T, f, g, obj = gw.solve_ugw(X, Y, _to_dev(torch, u), _to_dev(torch, v), 0.5, 0.01, 0, 10)
    torch.cuda.synchronize()
    T0 = np.outer(u, v) / math.sqrt(u.sum() * v.sum())
    assert err(T.cpu().numpy(), T0) <= TOL
    assert not f.abs().sum().item() and not g.abs().sum().item()
    U0, R0 = O.objective_ugw(ogrid(X), ogrid(Y), T0, u, v, 0.5, 0.01)
    o = obj.cpu().numpy()
    assert abs(o[0] - U0) <= TOL * abs(U0) and abs(o[1] - R0) <= TOL * abs(R0)


def test_solve_ugw_n1024_in_full():
    gw, torch = _gw()
    n = 1024
    X = gw.unit_grid((n,), 1)
    rng = inputs.rng_for(954)
    u, v = inputs.gauss_mixture_1d(n, rng), 1.3 * inputs.gauss_mixture_1d(n, rng)
    T0, f0, g0, (U0, _) = O.solve_ugw(ogrid(X), ogrid(X), u, v, 1.0, 0.005, 2, 20)
    T, f, g, obj = gw.solve_ugw(X, X, _to_dev(torch, u), _to_dev(torch, v), 1.0, 0.005, 2, 20)
    torch.cuda.synchronize()
    assert err(T.cpu().numpy(), T0) <= TOL
    assert abs(obj.cpu().numpy()[0] - U0) <= TOL * abs(U0)


def _random_uot_case(c):
    """Seeded random shape, parameters, costs and measures (some zero-mass
    rows and columns) for the sweep below."""
    rng = inputs.rng_for(955, c)
    M = int(rng.integers(1, 700))
    N = int(rng.choice([int(rng.integers(1, 300)), int(rng.integers(300, 2049)),
                        int(rng.integers(2049, 4097))]))
    rho, eps = float(10 ** rng.uniform(-1.3, 1.3)), float(10 ** rng.uniform(-3.5, -1))
    shift, scale = float(rng.uniform(-0.5, 0.5)), float(10 ** rng.uniform(-1, 0.7))
    iters = int(rng.integers(2, 9))
    C = rng.uniform(0, scale, (M, N))
    u, v = rng.uniform(0.0, 2.0 / M, M), rng.uniform(0.0, 3.0 / N, N)
    if M > 3:
        u[rng.choice(M, size=max(1, M // 10), replace=False)] = 0.0
    if N > 3 and rng.uniform() < 0.7:
        v[rng.choice(N, size=max(1, N // 10), replace=False)] = 0.0
    return C, u, v, rho, eps, shift, iters


@pytest.mark.parametrize("c", range(12))
def test_uot_sinkhorn_random_cases_match_oracle(c):
    """A seeded sweep over shapes (rows of 1-4096 entries), rho, eps, cost
    scales and shifts, with zero-mass entries: both pass kinds of the
    one-pass update under parameters no hand-picked case fixes."""
    gw, torch = _gw()
    C, u, v, rho, eps, shift, iters = _random_uot_case(c)
    M, N = C.shape
    print(f"uot random case {c}: M={M} N={N} rho={rho:.3g} eps={eps:.3g} shift={shift:.2f}", flush=True)
    f0, g0 = O.uot_sinkhorn(C + shift, u, v, rho, eps, iters)
    T0 = O.uot_plan(C + shift, f0, g0, u, v, eps)
    d = lambda a: _to_dev(torch, a)
    f, g, T = gw.uot_sinkhorn(d(C), d(u), d(v), rho, eps, iters, c_shift=shift, plan=True)
    torch.cuda.synchronize()
    fin = np.isfinite(f0)
    assert np.array_equal(np.isfinite(f.cpu().numpy()), fin)
    assert err(f.cpu().numpy()[fin], f0[fin]) <= TOL
    assert err(g.cpu().numpy(), g0) <= TOL
    assert err(T.cpu().numpy(), T0) <= TOL


def test_uot_sinkhorn_n4096_in_full():
    """The unbalanced Sinkhorn at the UGW workload's size and launch shape
    (rows of 4096 entries, shifted passes after the first): 3-Gaussian-mixture
    measures of mass 1 and 1.5, cost (x_i - y_p)^2 on the [0,1] grid,
    eps = 2e-3, 20 iterations; f, g and the plan in full."""
    gw, torch = _gw()
    n = 4096
    print(f"uot full n={n}", flush=True)
    rng = inputs.rng_for(13, n)
    u, v = inputs.gauss_mixture_1d(n, rng), 1.5 * inputs.gauss_mixture_1d(n, rng)
    x = np.arange(n) / (n - 1)
    C = (x[:, None] - x[None, :]) ** 2
    f0, g0 = O.uot_sinkhorn(C, u, v, 1.0, 2e-3, 20)
    T0 = O.uot_plan(C, f0, g0, u, v, 2e-3)
    d = lambda a: _to_dev(torch, a)
    f, g, T = gw.uot_sinkhorn(d(C), d(u), d(v), 1.0, 2e-3, 20, plan=True)
    torch.cuda.synchronize()
    assert err(f.cpu().numpy(), f0) <= TOL
    assert err(g.cpu().numpy(), g0) <= TOL
    assert err(T.cpu().numpy(), T0) <= TOL


def test_ugw_rejects_bad_arguments():
    gw, torch = _gw()
    X = gw.unit_grid((4,), 1)
    z = torch.full((4,), 0.25, dtype=torch.float64, device="cuda")
    for rho, eps in ((0.0, 0.1), (1.0, 0.0), (float("nan"), 0.1)):
        with pytest.raises(gw.GWError):
            gw.solve_ugw(X, X, z, z, rho, eps, 1, 1)
        with pytest.raises(gw.GWError):
            gw.uot_sinkhorn(torch.zeros((4, 4), dtype=torch.float64, device="cuda"), z, z, rho,
                            eps, 1)


def test_ugw_empty_measure_flags_numeric_status():
    """u = 0 has no plan to rescale: the non-finite step is reported through the
    workspace status (GW_ENUMERIC), not silently returned."""
    gw, torch = _gw()
    X = gw.unit_grid((16,), 1)
    u = torch.zeros(16, dtype=torch.float64, device="cuda")
    v = torch.full((16,), 1 / 16, dtype=torch.float64, device="cuda")
    ws = gw.workspace(gw.workspace_bytes(X, X, gw.PATH_FAST_F64, gw.OP_SOLVE_UGW), "cuda",
                      key="ugw_status")
    gw.solve_ugw(X, X, u, v, 1.0, 0.05, 2, 5, ws=ws)
    with pytest.raises(gw.GWError) as e:
        gw.check_status(ws)
    assert e.value.status == gw.GW_ENUMERIC
