"""GPU parity: every gw_* call through the C ABI against the CPU oracle.

Tolerance for FP64 paths: err(X) = max|X - X*| / max|X*| <= 1e-10; bit-exact
where every intermediate value is an integer below 2^53 (impulse and integer
inputs)."""
import math

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


def _to_dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def err(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(x)), "non-finite pattern differs"
    if not fin.any():
        return 0.0
    scale = np.max(np.abs(ref[fin]))
    return float(np.max(np.abs(x[fin] - ref[fin])) / (scale if scale > 0 else 1.0))


def ogrid(g):
    return O.Grid(tuple(g.shape), g.h, g.k, g.metric)


def _grad(gw, torch, X, Y, p, q, T, path="fast"):
    G = gw.grad(X, Y, _to_dev(torch, p), _to_dev(torch, q), _to_dev(torch, T), path=path)
    torch.cuda.synchronize()
    return G.cpu().numpy()


# ------------------------------------------------------------------ gradient

GRAD_1D = [(1, 1, 1, 1), (5, 7, 1, 2), (64, 64, 2, 2), (65, 63, 1, 1), (130, 70, 3, 1),
           (200, 300, 2, 3), (257, 129, 4, 4), (333, 64, 2, 1)]


@pytest.mark.parametrize("M,N,kx,ky", GRAD_1D)
@pytest.mark.parametrize("path", ["fast", "dense"])
def test_grad_1d_matches_oracle(M, N, kx, ky, path):
    gw, torch = _gw()
    print(f"grad 1d {path} M={M} N={N} kx={kx} ky={ky}", flush=True)
    rng = inputs.rng_for(201, M, N, kx, ky)
    X, Y = gw.unit_grid((M,), kx), gw.unit_grid((N,), ky)
    T = inputs.random_plan(M, N, rng)
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    ref = O.grad_dense(ogrid(X), ogrid(Y), p, q, T)
    G = _grad(gw, torch, X, Y, p, q, T, path)
    assert err(G, ref) <= TOL


def _random_grid_spec(rng, npts=800):
    """A seeded random grid of at most npts points: 1D, 2D (sides up to
    npts / 10) or 3D, k in 1..4 or squared Euclidean."""
    nd = int(rng.choice([1, 2, 3], p=[0.4, 0.4, 0.2]))
    if nd == 1:
        shape = (int(rng.integers(1, npts + 1)),)
    elif nd == 2:
        H = int(rng.integers(1, npts // 10 + 1))
        shape = (H, int(rng.integers(1, npts // H + 1)))
    else:
        side = int(round(npts ** (1.0 / 3.0)))
        shape = tuple(int(rng.integers(1, side + 1)) for _ in range(3))
    if rng.uniform() < 0.25:
        return shape, 2, 1
    return shape, int(rng.integers(1, 5)), 0


@pytest.mark.parametrize("c", range(16))
def test_grad_random_cases_match_oracle(c):
    """A seeded sweep over pairs of 1D, 2D and 3D grids (mixed pairs, ragged
    tiles, k = 1..4, both metrics), random plans and marginals; 1D pairs also
    on the dense path."""
    gw, torch = _gw()
    rng = inputs.rng_for(208, c)
    (sx, kx, mx), (sy, ky, my) = _random_grid_spec(rng), _random_grid_spec(rng)
    X, Y = gw.unit_grid(sx, kx, mx), gw.unit_grid(sy, ky, my)
    path = "dense" if len(sx) == 1 and len(sy) == 1 and rng.uniform() < 0.5 else "fast"
    print(f"grad random case {c}: {sx} k{kx} m{mx} x {sy} k{ky} m{my} {path}", flush=True)
    T = inputs.random_plan(X.size, Y.size, rng)
    p, q = inputs.dirichlet(X.size, rng), inputs.dirichlet(Y.size, rng)
    ref = O.grad_dense(ogrid(X), ogrid(Y), p, q, T)
    G = _grad(gw, torch, X, Y, p, q, T, path)
    assert err(G, ref) <= TOL


@pytest.mark.parametrize("M,N,kx,ky", [(97, 64, 1, 2), (64, 100, 2, 2), (129, 31, 2, 1)])
@pytest.mark.parametrize("path", ["fast", "dense"])
def test_grad_1d_integer_inputs_bit_exact(M, N, kx, ky, path):
    gw, torch = _gw()
    rng = inputs.rng_for(202, M, N)
    X, Y = gw.Grid((M,), 1.0, kx), gw.Grid((N,), 1.0, ky)
    T = inputs.integer_plan(M, N, rng)
    p = rng.integers(0, 5, size=M).astype(np.float64)
    q = rng.integers(0, 5, size=N).astype(np.float64)
    ref = O.grad_dense(ogrid(X), ogrid(Y), p, q, T)
    G = _grad(gw, torch, X, Y, p, q, T, path)
    assert np.array_equal(G, ref)


@pytest.mark.parametrize("shape,k,metric", [((50,), 2, 0), ((6, 7), 2, 0), ((5, 5), 2, 1)])
def test_impulse_bit_exact(shape, k, metric):
    gw, torch = _gw()
    X = gw.Grid(shape, 1.0, k, metric)
    D = O.integer_distance(ogrid(X)).astype(np.float64)
    n = X.size
    for j, q_ in [(0, n - 1), (n // 2, 1), (3, 3)]:
        T = np.zeros((n, n)); T[j, q_] = 1.0
        p = np.zeros(n); p[j] = 1.0
        q = np.zeros(n); q[q_] = 1.0
        ref = (D[:, j][:, None] - D[q_, :][None, :]) ** 2
        paths = ["fast", "dense"] if len(shape) == 1 else ["fast"]
        for path in paths:
            assert np.array_equal(_grad(gw, torch, X, X, p, q, T, path), ref)


GRAD_2D = [
    ((8, 8), 2, 1, (8, 8), 2, 1),      # SQEUCLID, separable
    ((7, 9), 1, 0, (5, 6), 1, 0),      # l1, k = 1, separable
    ((6, 5), 2, 0, (4, 7), 2, 0),      # l1^2: generic
    ((5, 5), 3, 0, (5, 5), 3, 0),      # l1^3: generic
    ((6, 6), 2, 1, (40,), 2, 0),       # mixed 2D x 1D: generic
    ((33,), 1, 0, (5, 4), 2, 1),       # mixed 1D x 2D
    ((16, 16), 2, 1, (12, 20), 2, 1),  # SQEUCLID H != W
    ((4, 6), 4, 0, (5, 3), 4, 0),      # l1^4: nine separable constant-term terms
    ((64, 64), 2, 0, (17, 40), 3, 0),  # l1^k image operator: a full 64 x 64 tile, a padded one
    ((1, 50), 2, 0, (63, 1), 4, 0),    # image operator on one-line images
    ((20, 64), 3, 0, (64, 9), 2, 0),   # image operator, H != W at the tile edge
    ((3, 70), 2, 1, (70, 2), 2, 1),    # SQEUCLID, image sides beyond one wave
]


@pytest.mark.parametrize("sx,kx,mx,sy,ky,my", GRAD_2D)
def test_grad_2d_matches_oracle(sx, kx, mx, sy, ky, my):
    gw, torch = _gw()
    print(f"grad 2d {sx} k{kx} m{mx} x {sy} k{ky} m{my}", flush=True)
    X, Y = gw.unit_grid(sx, kx, mx), gw.unit_grid(sy, ky, my)
    rng = inputs.rng_for(203, X.size, Y.size)
    T = inputs.random_plan(X.size, Y.size, rng)
    p, q = inputs.dirichlet(X.size, rng), inputs.dirichlet(Y.size, rng)
    ref = O.grad_dense(ogrid(X), ogrid(Y), p, q, T)
    assert err(_grad(gw, torch, X, Y, p, q, T), ref) <= TOL


def test_grad_deterministic():
    gw, torch = _gw()
    X = gw.unit_grid((300,), 2)
    rng = inputs.rng_for(204)
    T = _to_dev(torch, inputs.random_plan(300, 300, rng))
    p = _to_dev(torch, inputs.dirichlet(300, rng))
    for path in ("fast", "dense"):
        a = gw.grad(X, X, p, p, T, path=path).clone()
        b = gw.grad(X, X, p, p, T, path=path).clone()
        torch.cuda.synchronize()
        assert torch.equal(a, b)


# ------------------------------------------------------------------- Sinkhorn

# one case per row-pass length class (N <= 256, 512, 1024, 2048, 3072, 4096,
# 6144, 8192, 9216, 12288, 16384), bands of one and of several rows
SK_CASES = [(1, 1, 0.1, 3), (37, 29, 0.05, 1), (100, 130, 0.01, 37), (300, 257, 1e-3, 20),
            (64, 1000, 2e-3, 10), (70, 2000, 3e-3, 6), (600, 2500, 2e-3, 4),
            (513, 4100, 5e-3, 5), (200, 4096, 1e-3, 4), (70, 5000, 3e-3, 5),
            (33, 7000, 1e-3, 4), (600, 9216, 2e-3, 3), (40, 9000, 2e-3, 4),
            (25, 12000, 5e-3, 3), (300, 12288, 1e-3, 3), (19, 16384, 1e-3, 3)]


@pytest.mark.parametrize("M,N,eps,iters", SK_CASES)
def test_sinkhorn_matches_oracle(M, N, eps, iters):
    gw, torch = _gw()
    print(f"sinkhorn M={M} N={N} eps={eps} iters={iters}", flush=True)
    rng = inputs.rng_for(205, M, N)
    C = rng.uniform(0, 2, size=(M, N))
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    f0, g0 = O.sinkhorn(2.0 * C, p, q, eps, iters)
    P0 = O.plan(2.0 * C, f0, g0, eps)
    f, g, T = gw.sinkhorn(_to_dev(torch, C), _to_dev(torch, p), _to_dev(torch, q), eps, iters,
                          c_scale=2.0, plan=True)
    torch.cuda.synchronize()
    assert err(f.cpu().numpy(), f0) <= TOL
    assert err(g.cpu().numpy(), g0) <= TOL
    assert err(T.cpu().numpy(), P0) <= TOL


def _random_sk_case(c):
    """Seeded random shape (rows of 1-24000 entries), eps, cost scale and
    marginals (some zero-mass entries), iteration count and start."""
    rng = inputs.rng_for(207, c)
    M = int(rng.integers(1, 700))
    N = int(rng.choice([int(rng.integers(1, 300)), int(rng.integers(300, 4097)),
                        int(rng.integers(4097, 16385)), int(rng.integers(16385, 24000))],
                       p=[0.25, 0.35, 0.3, 0.1]))
    eps, scale = float(10 ** rng.uniform(-3.3, -1)), float(10 ** rng.uniform(-1, 0.7))
    iters = int(rng.integers(2, 9))
    C = rng.uniform(0, scale, (M, N))
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    if M > 3 and rng.uniform() < 0.5:
        p[rng.choice(M, size=max(1, M // 20), replace=False)] = 0.0
        p /= p.sum()
    if N > 3 and rng.uniform() < 0.5:
        q[rng.choice(N, size=max(1, N // 20), replace=False)] = 0.0
        q /= q.sum()
    warm = bool(rng.uniform() < 0.3)
    return C, p, q, eps, iters, warm


@pytest.mark.parametrize("c", range(12))
def test_sinkhorn_random_cases_match_oracle(c):
    """A seeded sweep over shapes, eps, cost scales, zero-mass entries and
    warm starts (from the oracle's potentials after two iterations): the row
    pass classes, both pass kinds and the wide-row slabs under parameters no
    hand-picked case fixes."""
    gw, torch = _gw()
    C, p, q, eps, iters, warm = _random_sk_case(c)
    M, N = C.shape
    print(f"sinkhorn random case {c}: M={M} N={N} eps={eps:.3g} iters={iters} warm={warm}",
          flush=True)
    d = lambda a: _to_dev(torch, a)
    if warm:
        fw, gw0 = O.sinkhorn(C, p, q, eps, 2)
        f0, g0 = O.sinkhorn(C, p, q, eps, iters, fw, gw0)
        f, g, T = gw.sinkhorn(d(C), d(p), d(q), eps, iters, f=d(fw), g=d(gw0), plan=True)
    else:
        f0, g0 = O.sinkhorn(C, p, q, eps, iters)
        f, g, T = gw.sinkhorn(d(C), d(p), d(q), eps, iters, plan=True)
    torch.cuda.synchronize()
    assert err(f.cpu().numpy(), f0) <= TOL
    assert err(g.cpu().numpy(), g0) <= TOL
    assert err(T.cpu().numpy(), O.plan(C, f0, g0, eps)) <= TOL


def test_sinkhorn_extreme_ratio_exact_then_shifted_passes():
    """C/eps up to 7000: the first update moves g by more than 600 eps (the
    next pass takes exact maxima), later ones by a few eps (shifted passes)."""
    gw, torch = _gw()
    rng = inputs.rng_for(206)
    M, N = 90, 70
    C = rng.uniform(0, 4, size=(M, N))
    C[:, 5] += 3.0
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    eps = 1e-3
    f0, g0 = O.sinkhorn(C, p, q, eps, 6)
    f, g, T = gw.sinkhorn(_to_dev(torch, C), _to_dev(torch, p), _to_dev(torch, q), eps, 6, plan=True)
    torch.cuda.synchronize()
    assert err(f.cpu().numpy(), f0) <= TOL
    assert err(g.cpu().numpy(), g0) <= TOL
    assert err(T.cpu().numpy(), O.plan(C, f0, g0, eps)) <= TOL


def test_sinkhorn_zero_mass_and_extreme_ratio():
    gw, torch = _gw()
    rng = inputs.rng_for(206)
    M, N = 90, 70
    C = rng.uniform(0, 4, size=(M, N))        # C/eps up to 4000
    C[:, 5] += 3.0                            # a column no row favours
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    p[[0, 17]] = 0.0; p /= p.sum()
    q[[3, 69]] = 0.0; q /= q.sum()
    eps = 1e-3
    f0, g0 = O.sinkhorn(C, p, q, eps, 25)
    f, g, T = gw.sinkhorn(_to_dev(torch, C), _to_dev(torch, p), _to_dev(torch, q), eps, 25, plan=True)
    torch.cuda.synchronize()
    f, g, T = f.cpu().numpy(), g.cpu().numpy(), T.cpu().numpy()
    assert np.isneginf(f[0]) and np.isneginf(f[17]) and np.isneginf(g[3]) and np.isneginf(g[69])
    assert err(f, f0) <= TOL and err(g, g0) <= TOL
    assert err(T, O.plan(C, f0, g0, eps)) <= TOL
    assert np.all(T[0] == 0) and np.all(T[:, 3] == 0)


# rows of more than 16384 entries: slabs of 8192 columns, two passes per iteration
WIDE_CASES = [(40, 20000, 2e-3, 3), (70, 16385, 1e-3, 4), (300, 33000, 5e-3, 3),
              (3, 65535, 5e-3, 2)]


@pytest.mark.parametrize("M,N,eps,iters", WIDE_CASES)
def test_sinkhorn_wide_rows_match_oracle(M, N, eps, iters):
    gw, torch = _gw()
    print(f"sinkhorn wide rows M={M} N={N} eps={eps} iters={iters}", flush=True)
    rng = inputs.rng_for(212, M, N)
    C = rng.uniform(0, 2, size=(M, N))
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    p[M // 2] = 0.0; p /= p.sum()
    q[[7, N - 2]] = 0.0; q /= q.sum()
    f0, g0 = O.sinkhorn(2.0 * C, p, q, eps, iters)
    f, g, T = gw.sinkhorn(_to_dev(torch, C), _to_dev(torch, p), _to_dev(torch, q), eps, iters,
                          c_scale=2.0, plan=True)
    torch.cuda.synchronize()
    assert err(f.cpu().numpy(), f0) <= TOL
    assert err(g.cpu().numpy(), g0) <= TOL
    assert err(T.cpu().numpy(), O.plan(2.0 * C, f0, g0, eps)) <= TOL


def test_sinkhorn_wide_rows_warm_start():
    gw, torch = _gw()
    rng = inputs.rng_for(213)
    M, N = 50, 17000
    C = rng.uniform(0, 1, size=(M, N))
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    f1, g1 = O.sinkhorn(C, p, q, 0.02, 3)
    f2, g2 = O.sinkhorn(C, p, q, 0.02, 2, f1, g1)
    fd, gd = gw.sinkhorn(_to_dev(torch, C), _to_dev(torch, p), _to_dev(torch, q), 0.02, 3)
    fd, gd = gw.sinkhorn(_to_dev(torch, C), _to_dev(torch, p), _to_dev(torch, q), 0.02, 2, f=fd, g=gd)
    torch.cuda.synchronize()
    assert err(fd.cpu().numpy(), f2) <= TOL and err(gd.cpu().numpy(), g2) <= TOL


def _max_distance(G):
    """The largest distance on a grid: (h sum (side - 1))^k, or h^2 sum
    (side - 1)^2 for squared Euclidean."""
    ext = [s - 1 for s in G.shape]
    if G.metric == 1:
        return G.h * G.h * sum(e * e for e in ext)
    return (G.h * sum(ext)) ** G.k


@pytest.mark.parametrize("c", range(8))
def test_solve_random_cases_match_oracle(c):
    """A seeded sweep of short solves over random grid pairs (1D, 2D, 3D,
    mixed; k = 1..4, both metrics), Dirichlet marginals, eps, outer and inner
    counts, cold or warm Sinkhorn starts, FAST or (1D pairs) dense: T, f, g
    and both objectives."""
    gw, torch = _gw()
    rng = inputs.rng_for(215, c)
    (sx, kx, mx), (sy, ky, my) = _random_grid_spec(rng, 300), _random_grid_spec(rng, 300)
    X, Y = gw.unit_grid(sx, kx, mx), gw.unit_grid(sy, ky, my)
    path = "dense" if len(sx) == 1 and len(sy) == 1 and rng.uniform() < 0.5 else "fast"
    # eps relative to the squared largest distance (the cost's scale), so that
    # C/eps stays in the thousands: far beyond, the plan's exponentials turn
    # rounding in C into relative errors above the tolerance on any FP64 path
    dmax = max(_max_distance(X), _max_distance(Y))
    eps = float(10 ** rng.uniform(-3.5, -1.8)) * (dmax * dmax if dmax > 0 else 1.0)
    outer, inner = int(rng.integers(1, 4)), int(rng.integers(5, 31))
    warm = bool(rng.uniform() < 0.3)
    p, q = inputs.dirichlet(X.size, rng), inputs.dirichlet(Y.size, rng)
    print(f"solve random case {c}: {sx} k{kx} m{mx} x {sy} k{ky} m{my} eps={eps:.3g} "
          f"{outer}x{inner} warm={warm} {path}", flush=True)
    T0, f0, g0, (E0, R0) = O.solve(ogrid(X), ogrid(Y), p, q, eps, outer, inner, warm=warm)
    T, f, g, obj = gw.solve(X, Y, _to_dev(torch, p), _to_dev(torch, q), eps, outer, inner,
                            path=path, warm=warm)
    torch.cuda.synchronize()
    assert err(T.cpu().numpy(), T0) <= TOL
    assert err(f.cpu().numpy(), f0) <= TOL
    assert err(g.cpu().numpy(), g0) <= TOL
    o = obj.cpu().numpy()
    assert abs(o[0] - E0) <= TOL * abs(E0)
    assert abs(o[1] - R0) <= TOL * max(abs(R0), abs(E0))


def test_solve_wide_rows_match_oracle():
    """A solve whose Y grid has more than 16384 points (the Sinkhorn calls run
    the slab path), against the oracle with its recursion gradient."""
    gw, torch = _gw()
    X, Y = gw.unit_grid((200,), 2), gw.unit_grid((17000,), 1)
    rng = inputs.rng_for(214)
    p, q = inputs.gauss_mixture_1d(200, rng), inputs.gauss_mixture_1d(17000, rng)
    eps, outer, inner = 5e-3, 2, 6
    T0, f0, g0, (E0, R0) = O.solve(ogrid(X), ogrid(Y), p, q, eps, outer, inner, gradient="pascal")
    T, f, g, obj = gw.solve(X, Y, _to_dev(torch, p), _to_dev(torch, q), eps, outer, inner)
    torch.cuda.synchronize()
    assert err(T.cpu().numpy(), T0) <= TOL
    assert err(f.cpu().numpy(), f0) <= TOL and err(g.cpu().numpy(), g0) <= TOL
    o = obj.cpu().numpy()
    assert abs(o[0] - E0) <= TOL * abs(E0)


def _tail_marginal(n, rng, lo):
    """Normalised Gaussian bump with tails hundreds of decades below its peak
    (the decay rate is set by `lo`), and two exact zeros."""
    x = np.linspace(-1.0, 1.0, n)
    c = rng.uniform(-0.3, 0.3)
    w = np.exp(-((x - c) ** 2) * (-lo * np.log(10.0)) / 1.3 ** 2)
    w[[n // 7, n - 3]] = 0.0
    return w / w.sum()


@pytest.mark.parametrize("M,N,lo", [(300, 4096, -320), (129, 1000, -250), (70, 3000, -120)])
def test_sinkhorn_tiny_marginal_entries(M, N, lo):
    """Marginal entries from 1 down to subnormal values: columns whose q_p is
    below 2^-101 get a frame 2^kq_p in the fast passes, rows with tiny p_i
    weights far from 1; every potential and plan entry against the oracle."""
    gw, torch = _gw()
    print(f"sinkhorn tiny marginals M={M} N={N} lo={lo}", flush=True)
    rng = inputs.rng_for(211, M, N)
    C = rng.uniform(0, 1, size=(M, N))
    p, q = _tail_marginal(M, rng, lo), _tail_marginal(N, rng, lo)
    assert np.any((q > 0) & (q < 2.0 ** -101))  # columns with a frame
    eps, iters = 5e-3, 8
    f0, g0 = O.sinkhorn(2.0 * C, p, q, eps, iters)
    f, g, T = gw.sinkhorn(_to_dev(torch, C), _to_dev(torch, p), _to_dev(torch, q), eps, iters,
                          c_scale=2.0, plan=True)
    torch.cuda.synchronize()
    assert err(f.cpu().numpy(), f0) <= TOL
    assert err(g.cpu().numpy(), g0) <= TOL
    assert err(T.cpu().numpy(), O.plan(2.0 * C, f0, g0, eps)) <= TOL


def test_sinkhorn_warm_start_and_zero_iterations():
    gw, torch = _gw()
    rng = inputs.rng_for(207)
    M, N = 50, 60
    C = rng.uniform(0, 1, size=(M, N))
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    f1, g1 = O.sinkhorn(C, p, q, 0.02, 7)
    f2, g2 = O.sinkhorn(C, p, q, 0.02, 5, f1, g1)
    fd, gd = gw.sinkhorn(_to_dev(torch, C), _to_dev(torch, p), _to_dev(torch, q), 0.02, 7)
    fd, gd = gw.sinkhorn(_to_dev(torch, C), _to_dev(torch, p), _to_dev(torch, q), 0.02, 5, f=fd, g=gd)
    torch.cuda.synchronize()
    assert err(fd.cpu().numpy(), f2) <= TOL and err(gd.cpu().numpy(), g2) <= TOL
    f0, g0, T0 = gw.sinkhorn(_to_dev(torch, C), _to_dev(torch, p), _to_dev(torch, q), 0.02, 0, plan=True)
    torch.cuda.synchronize()
    assert np.all(f0.cpu().numpy() == 0) and np.all(g0.cpu().numpy() == 0)
    assert err(T0.cpu().numpy(), np.exp(-C / 0.02)) <= TOL


# ---------------------------------------------------------------------- solve

SOLVE_CASES = [
    ((64,), 2, 0, (64,), 2, 0, 5e-3, 5, 20, "fast"),
    ((64,), 2, 0, (64,), 2, 0, 5e-3, 5, 20, "dense"),
    ((100,), 1, 0, (80,), 3, 0, 2e-3, 4, 30, "fast"),
    ((6, 6), 2, 1, (6, 6), 2, 1, 2e-3, 3, 20, "fast"),
    ((5, 6), 2, 0, (7, 4), 1, 0, 5e-3, 3, 20, "fast"),
]


@pytest.mark.parametrize("sx,kx,mx,sy,ky,my,eps,outer,inner,path", SOLVE_CASES)
def test_solve_matches_oracle(sx, kx, mx, sy, ky, my, eps, outer, inner, path):
    gw, torch = _gw()
    print(f"solve {sx} {sy} eps={eps} {outer}x{inner} {path}", flush=True)
    X, Y = gw.unit_grid(sx, kx, mx), gw.unit_grid(sy, ky, my)
    rng = inputs.rng_for(208, X.size, Y.size)
    if len(sx) == 1:
        p = inputs.gauss_mixture_1d(X.size, rng)
    else:
        p = inputs.blobs_2d(sx[0], sx[1], rng, floor=1e-6)
    if len(sy) == 1:
        q = inputs.gauss_mixture_1d(Y.size, rng)
    else:
        q = inputs.blobs_2d(sy[0], sy[1], rng, floor=1e-6)
    T0, f0, g0, (E0, R0) = O.solve(ogrid(X), ogrid(Y), p, q, eps, outer, inner)
    T, f, g, obj = gw.solve(X, Y, _to_dev(torch, p), _to_dev(torch, q), eps, outer, inner, path=path)
    torch.cuda.synchronize()
    assert err(T.cpu().numpy(), T0) <= TOL
    assert err(f.cpu().numpy(), f0) <= TOL
    assert err(g.cpu().numpy(), g0) <= TOL
    o = obj.cpu().numpy()
    assert abs(o[0] - E0) <= TOL * abs(E0)
    assert abs(o[1] - R0) <= TOL * max(abs(R0), abs(E0))


def test_objective_zero_at_identity_coupling():
    gw, torch = _gw()
    n = 64
    X = gw.Grid((n,), 1.0, 2)
    obj = gw.objective(X, X, _to_dev(torch, np.eye(n) / n), 0.0)
    torch.cuda.synchronize()
    assert obj.cpu().numpy()[0] == 0.0


def test_objective_matches_oracle():
    gw, torch = _gw()
    rng = inputs.rng_for(209)
    X, Y = gw.unit_grid((120,), 2), gw.unit_grid((90,), 1)
    T = inputs.random_plan(120, 90, rng)
    E0, R0 = O.objective(ogrid(X), ogrid(Y), T, 0.01)
    o = gw.objective(X, Y, _to_dev(torch, T), 0.01).cpu().numpy()
    assert abs(o[0] - E0) <= TOL * abs(E0) and abs(o[1] - R0) <= TOL * abs(E0)


def test_invalid_call_raises():
    gw, torch = _gw()
    X = gw.unit_grid((16,), 1)
    T = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    p = torch.full((16,), 1 / 16, dtype=torch.float64, device="cuda")
    with pytest.raises(gw.GWError):
        gw.grad(X, X, p, p, T, out=T)          # output overlaps input
    with pytest.raises(gw.GWError):
        gw.sinkhorn(T, p, p, -1.0, 3)


# ------------------------------------------------------------ precision study

LP_PATHS = {
    # path: (unit roundoff of the operands, FP32-accumulated chunk length or None = whole K)
    "dense_f32": (2.0 ** -24, None),
    "dense_bf16": (2.0 ** -8, None),
    "dense_f32_split": (2.0 ** -48, 4),
    "dense_bf16_split": (2.0 ** -16, 256),
}


def lp_bound(path, K):
    """A-priori relative bound on the bilinear part for non-negative operands:
    4 operand roundings (T, D_Y, A, D_X) plus FP32 accumulation over the
    accumulated chunk in each of the two products (gamma_K = K u / (1 - K u))."""
    u_in, chunk = LP_PATHS[path]
    u32 = 2.0 ** -24
    kk = K if chunk is None else min(chunk, K)
    gamma = kk * u32 / (1 - kk * u32)
    return 4 * u_in + 2 * gamma + 1e-12


@pytest.mark.parametrize("n,k", [(200, 1), (1000, 2), (777, 3)])
def test_dense_low_precision_within_bound(n, k):
    gw, torch = _gw()
    rng = inputs.rng_for(210, n, k)
    X = gw.unit_grid((n,), k)
    T = inputs.peaked_plan(n, n, rng)
    p, q = inputs.dirichlet(n, rng), inputs.dirichlet(n, rng)
    G0 = O.grad_dense(ogrid(X), ogrid(X), p, q, T)
    c1, c2 = O.const_terms(O.cost_matrix(ogrid(X)), O.cost_matrix(ogrid(X)), p, q)
    bil = c1[:, None] + c2[None, :] - G0           # = 2 D_X T D_Y
    errs = {}
    for path in LP_PATHS:
        G = _grad(gw, torch, X, X, p, q, T, path)
        e = float(np.max(np.abs(G - G0)) / np.max(np.abs(bil)))
        errs[path] = e
        print(f"{path} n={n} k={k} err_bilinear={e:.3e} bound={lp_bound(path, n):.3e}", flush=True)
        assert e <= lp_bound(path, n)
    assert errs["dense_f32_split"] < errs["dense_f32"]
    assert errs["dense_bf16_split"] < errs["dense_bf16"]


@pytest.mark.parametrize("sx,kx,sy,ky", [((10, 12), 2, (9, 7), 3), ((64, 5), 2, (8, 64), 2)])
def test_grad_2d_image_operator_integer_bit_exact(sx, kx, sy, ky):
    """(l1)^k image operator on integer inputs (h = 1): every intermediate is an
    integer below 2^53, so the result equals the oracle's exactly."""
    gw, torch = _gw()
    X, Y = gw.Grid(sx, 1.0, kx), gw.Grid(sy, 1.0, ky)
    rng = inputs.rng_for(209, X.size, Y.size)
    T = inputs.integer_plan(X.size, Y.size, rng, hi=4)
    p = rng.integers(0, 3, size=X.size).astype(np.float64)
    q = rng.integers(0, 3, size=Y.size).astype(np.float64)
    ref = O.grad_dense(ogrid(X), ogrid(Y), p, q, T)
    assert np.max(np.abs(ref)) < 2.0 ** 53
    assert np.array_equal(_grad(gw, torch, X, Y, p, q, T), ref)
