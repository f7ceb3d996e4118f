"""GPU parity at the benchmark sizes, in the launch configurations bench.py
times: the FAST gradient at n = 4096 (k = 1, 2, 3) and n = 16384 (k = 2) on
sampled rows (each computed by the oracle from the plain definition), the 2D
64 x 64 gradient and one Sinkhorn call at n = 4096 in full, one outer step of
the n = 4096 solve in full, and properties of the whole 100 x 100 solve that
hold at any size.  Tolerance for FP64: relative 1e-10."""
import numpy as np
import pytest

from oracle import gw_oracle as O
from paper_2404_08970_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _gw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_08970_amd import gw
    return gw, torch


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _rel(x, ref):
    x, ref = np.asarray(x), np.asarray(ref)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(x)), "non-finite pattern differs"
    return float(np.max(np.abs(x[fin] - ref[fin])) / np.max(np.abs(ref[fin])))


def _bench_marginals(n, k):
    # the bench workload's keys: (2, side, k)
    return (inputs.gauss_mixture_1d(n, inputs.rng_for(2, 0, k)),
            inputs.gauss_mixture_1d(n, inputs.rng_for(2, 1, k)))


def _sample_rows(n):
    # ends, both sides of tile edges (64), a band edge of the Sinkhorn pass, the middle
    return np.unique(np.array([0, 1, 63, 64, 65, 127, 128, n // 2 - 1, n // 2, n - 65, n - 64,
                               n - 2, n - 1]))


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("plan", ["uniform", "peaked"])
def test_fast_grad_n4096_sampled_rows(k, plan):
    gw, torch = _gw()
    n = 4096
    print(f"fullsize grad n={n} k={k} plan={plan}", flush=True)
    p, q = _bench_marginals(n, k)
    rng = inputs.rng_for(600, k)
    T = inputs.random_plan(n, n, rng) if plan == "uniform" else inputs.peaked_plan(n, n, rng)
    X = gw.unit_grid((n,), k)
    G = gw.grad(X, X, _dev(torch, p), _dev(torch, q), _dev(torch, T), path="fast")
    rows = _sample_rows(n)
    Gs = G[torch.tensor(rows, device="cuda")].cpu().numpy()
    og = O.Grid((n,), X.h, k)
    ref = O.grad_rows(og, og, p, q, T, rows)
    assert _rel(Gs, ref) <= TOL


def test_fast_grad_n16384_sampled_rows():
    gw, torch = _gw()
    n, k = 16384, 2
    print(f"fullsize grad n={n} k={k}", flush=True)
    rng = inputs.rng_for(4, 2)
    p, q = inputs.dirichlet(n, rng), inputs.dirichlet(n, rng)
    T = inputs.random_plan(n, n, rng)
    X = gw.unit_grid((n,), k)
    Td = _dev(torch, T)
    G = gw.grad(X, X, _dev(torch, p), _dev(torch, q), Td, path="fast")
    rows = np.array([0, 64, 4095, 8191, 8192, 16319, 16383])
    Gs = G[torch.tensor(rows, device="cuda")].cpu().numpy()
    del G, Td
    og = O.Grid((n,), X.h, k)
    ref = O.grad_rows(og, og, p, q, T, rows, block=2048)
    assert _rel(Gs, ref) <= TOL


def test_fast_grad_2d_64x64_full():
    gw, torch = _gw()
    side = 64
    print("fullsize grad 2D 64x64 SQEUCLID", flush=True)
    X = gw.unit_grid((side, side), 2, gw.METRIC_SQEUCLID)
    p = inputs.blobs_2d(side, side, inputs.rng_for(3, 0), floor=1e-6)
    q = inputs.blobs_2d(side, side, inputs.rng_for(3, 1), floor=1e-6)
    T = inputs.peaked_plan(X.size, X.size, inputs.rng_for(601))
    G = gw.grad(X, X, _dev(torch, p), _dev(torch, q), _dev(torch, T), path="fast").cpu().numpy()
    og = O.Grid((side, side), X.h, 2, O.METRIC_SQEUCLID)
    assert _rel(G, O.grad_dense(og, og, p, q, T)) <= TOL


def test_sinkhorn_n4096_full():
    """One Sinkhorn call of the bench workload (cost 2G at T = p q^T, k = 2,
    eps = 1e-3), every potential and every plan entry."""
    gw, torch = _gw()
    n, k, eps, iters = 4096, 2, 1e-3, 6
    print(f"fullsize sinkhorn n={n} iters={iters}", flush=True)
    p, q = _bench_marginals(n, k)
    og = O.Grid((n,), 1 / (n - 1), k)
    C = 2.0 * O.grad_dense(og, og, p, q, np.outer(p, q))
    f, g, T = gw.sinkhorn(_dev(torch, C), _dev(torch, p), _dev(torch, q), eps, iters, plan=True)
    f0, g0 = O.sinkhorn(C, p, q, eps, iters)
    T0 = O.plan(C, f0, g0, eps)
    assert _rel(f.cpu().numpy(), f0) <= TOL
    assert _rel(g.cpu().numpy(), g0) <= TOL
    assert _rel(T.cpu().numpy(), T0) <= TOL


def test_sinkhorn_wide_n32768_full():
    """Rows of 32768 entries (two passes per iteration over slabs of 8192
    columns), 4096 rows, mixture marginals with underflowing tails, a seeded
    uniform cost: every potential and every plan entry."""
    gw, torch = _gw()
    M, N, k, eps, iters = 4096, 32768, 2, 1e-3, 3
    print(f"fullsize wide sinkhorn M={M} N={N} iters={iters}", flush=True)
    p = inputs.gauss_mixture_1d(M, inputs.rng_for(2, 0, k))
    q = inputs.gauss_mixture_1d(N, inputs.rng_for(2, 1, k))
    C = inputs.rng_for(601).uniform(0.0, 1.0, size=(M, N))
    f, g, T = gw.sinkhorn(_dev(torch, C), _dev(torch, p), _dev(torch, q), eps, iters, plan=True)
    torch.cuda.synchronize()
    f0, g0 = O.sinkhorn(C, p, q, eps, iters)
    assert _rel(f.cpu().numpy(), f0) <= TOL
    assert _rel(g.cpu().numpy(), g0) <= TOL
    assert _rel(T.cpu().numpy(), O.plan(C, f0, g0, eps)) <= TOL


def test_solve_n4096_one_outer_full():
    gw, torch = _gw()
    n, k, eps = 4096, 2, 1e-3
    print(f"fullsize solve n={n} outer=1 inner=5", flush=True)
    p, q = _bench_marginals(n, k)
    X = gw.unit_grid((n,), k)
    T, f, g, obj = gw.solve(X, X, _dev(torch, p), _dev(torch, q), eps, 1, 5, path="fast")
    og = O.Grid((n,), X.h, k)
    T0, f0, g0, obj0 = O.solve(og, og, p, q, eps, 1, 5)
    assert _rel(T.cpu().numpy(), T0) <= TOL
    assert _rel(f.cpu().numpy(), f0) <= TOL
    assert _rel(g.cpu().numpy(), g0) <= TOL
    o = obj.cpu().numpy()
    assert abs(o[0] - obj0[0]) <= TOL * abs(obj0[0])
    assert abs(o[1] - obj0[1]) <= TOL * max(abs(obj0[1]), abs(obj0[0]))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_solve_bench_config_properties(k):
    """The whole bench solve (n = 4096, 100 x 100, eps = 1e-3): the plan is
    non-negative and its column sums equal q (the last Sinkhorn update is on
    g); potentials are finite where the marginals are positive; the objective
    is finite and non-negative up to rounding.  The row-marginal error is
    printed (it depends on how far 100 iterations converge at this eps)."""
    gw, torch = _gw()
    n, eps = 4096, 1e-3
    print(f"fullsize solve properties n={n} k={k} 100x100", flush=True)
    p, q = _bench_marginals(n, k)
    X = gw.unit_grid((n,), k)
    pd, qd = _dev(torch, p), _dev(torch, q)
    T, f, g, obj = gw.solve(X, X, pd, qd, eps, 100, 100, path="fast")
    gw.check_status()
    assert bool((T >= 0).all())
    cols = T.sum(dim=0).cpu().numpy()
    rows = T.sum(dim=1).cpu().numpy()
    assert np.max(np.abs(cols - q)) <= 1e-12
    print(f"row marginal L1 error {np.sum(np.abs(rows - p)):.3e}", flush=True)
    fn, gn = f.cpu().numpy(), g.cpu().numpy()
    assert np.all(np.isfinite(fn[p > 0])) and np.all(np.isfinite(gn[q > 0]))
    o = obj.cpu().numpy()
    assert np.all(np.isfinite(o)) and o[0] >= -1e-12
