"""GPU parity of the tolerance-stopped Sinkhorn and solve against the oracle.

The stop decision compares a floating-point sum with tol; every case picks tol
in a clear gap of the oracle's violation trajectory, so both sides stop at the
same iteration, and then f, g, T match to the FP64 bar (1e-10 relative)."""
import numpy as np
import pytest

from oracle import gw_oracle as O
from paper_2404_08970_amd import inputs

from test_gpu_parity import TOL, _gw, _to_dev, err, ogrid

pytestmark = pytest.mark.gpu


def _check_errs(C, p, q, eps, every, checks, f0=None, g0=None, below=None):
    """The oracle's violation at checks 1..checks (iteration k * every), check
    by check: each call continues from the previous potentials, which is the
    same arithmetic as one longer call.  Stops early once a value <= below."""
    out = []
    f, g = f0, g0
    for _ in range(checks):
        f, g, _, e = O.sinkhorn_tol(C, p, q, eps, every, every, -1.0, f, g)
        out.append(e)
        if below is not None and e <= below:
            break
    return out


def _gap_tol(errs, start=2):
    """tol in the first clear gap (ratio < 0.9) from check `start` on."""
    for j in range(start, len(errs)):
        if errs[j] < 0.9 * errs[j - 1]:
            return (errs[j] * errs[j - 1]) ** 0.5, j + 1
    raise AssertionError("no gap in the violation trajectory")


CASES = [(37, 100, 0.05, 1), (64, 700, 0.02, 3), (20, 1500, 0.03, 2), (40, 3000, 0.02, 4),
         (33, 4096, 0.01, 5), (17, 5000, 0.03, 2), (12, 9000, 0.02, 3), (9, 16384, 0.05, 2)]


@pytest.mark.parametrize("M,N,eps,every", CASES)
def test_sinkhorn_tol_matches_oracle(M, N, eps, every):
    gw, torch = _gw()
    print(f"sinkhorn_tol M={M} N={N} eps={eps} every={every}", flush=True)
    rng = inputs.rng_for(910, M, N)
    C = rng.uniform(0, 1, size=(M, N))
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    errs = _check_errs(C, p, q, eps, every, 8)
    tol, kstop = _gap_tol(errs)
    f0, g0, k0, e0 = O.sinkhorn_tol(C, p, q, eps, 200, every, tol)
    assert k0 == kstop * every
    T0 = O.plan(C, f0, g0, eps)
    d = lambda a: _to_dev(torch, a)
    f, g, T, done, e = gw.sinkhorn_tol(d(C), d(p), d(q), eps, 200, every, tol, plan=True)
    torch.cuda.synchronize()
    assert int(done.item()) == k0
    assert abs(float(e.item()) - e0) <= TOL * e0
    assert err(f.cpu().numpy(), f0) <= TOL
    assert err(g.cpu().numpy(), g0) <= TOL
    assert err(T.cpu().numpy(), T0) <= TOL


def test_sinkhorn_tol_unmet_equals_fixed_count():
    gw, torch = _gw()
    rng = inputs.rng_for(911)
    C = _to_dev(torch, rng.uniform(0, 1, size=(50, 300)))
    p = _to_dev(torch, inputs.dirichlet(50, rng))
    q = _to_dev(torch, inputs.dirichlet(300, rng))
    f, g, done, e = gw.sinkhorn_tol(C, p, q, 0.02, 23, 4, 0.0)
    f2, g2 = gw.sinkhorn(C, p, q, 0.02, 23)
    torch.cuda.synchronize()
    assert int(done.item()) == 23 and float(e.item()) > 0.0
    assert torch.equal(f, f2) and torch.equal(g, g2)


def test_sinkhorn_tol_graph_replays_equal_eager():
    """Captured into a HIP graph the call waits for nothing on the host: every
    launch is recorded and the ones after the stop return at once.  Three
    replays, with eager Sinkhorn work between them, each equal the eager call
    bit for bit (potentials, plan, iterations done)."""
    gw, torch = _gw()
    rng = inputs.rng_for(915)
    M, N = 120, 900
    C = _to_dev(torch, rng.uniform(0, 1, size=(M, N)))
    p = _to_dev(torch, inputs.dirichlet(M, rng))
    q = _to_dev(torch, inputs.dirichlet(N, rng))
    f0, g0, T0, d0, _ = gw.sinkhorn_tol(C, p, q, 0.05, 200, 10, 1e-9, plan=True)
    torch.cuda.synchronize()
    n0 = int(d0.item())
    assert 0 < n0 < 200
    nb = gw.workspace_bytes(gw.unit_grid((M,), 1), gw.unit_grid((N,), 1), gw.PATH_FAST_F64,
                            gw.OP_SINKHORN)
    ws = gw.workspace(nb, "cuda", key="capture")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        f, g, T, d, _ = gw.sinkhorn_tol(C, p, q, 0.05, 200, 10, 1e-9, plan=True, ws=ws)
    for r in range(3):
        print(f"replay {r}", flush=True)
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(f, f0) and torch.equal(g, g0) and torch.equal(T, T0)
        assert int(d.item()) == n0
        gw.sinkhorn(C, p, q, 0.05, 7)  # eager work between the replays
        torch.cuda.synchronize()


def test_sinkhorn_tol_zero_mass_and_warm_start():
    gw, torch = _gw()
    M, N, eps, every = 30, 260, 0.03, 2
    rng = inputs.rng_for(912)
    C = rng.uniform(0, 1, size=(M, N))
    p, q = inputs.dirichlet(M, rng), inputs.dirichlet(N, rng)
    p[[0, 7]] = 0.0
    q[[3, 100, 259]] = 0.0
    p, q = p / p.sum(), q / q.sum()
    fw, gw0 = O.sinkhorn(C, p, q, eps, 3)
    errs = _check_errs(C, p, q, eps, every, 8, fw, gw0)
    tol, _ = _gap_tol(errs)
    f0, g0, k0, e0 = O.sinkhorn_tol(C, p, q, eps, 100, every, tol, fw, gw0)
    d = lambda a: _to_dev(torch, a)
    f, g, done, e = gw.sinkhorn_tol(d(C), d(p), d(q), eps, 100, every, tol, f=d(fw), g=d(gw0))
    torch.cuda.synchronize()
    assert int(done.item()) == k0
    assert err(f.cpu().numpy(), f0) <= TOL and err(g.cpu().numpy(), g0) <= TOL


def test_sinkhorn_tol_full_size_properties():
    """n = 4096 (the 1D bench size, k = 2 cost of a solve's first step): the
    stopped call equals gw_sinkhorn run for the iterations it reports, bitwise;
    its violation is <= tol and the check before it was above tol."""
    gw, torch = _gw()
    n, eps, every, cap = 4096, 1e-3, 10, 2000
    X = gw.unit_grid((n,), 2)
    rng = inputs.rng_for(2, n, 2)
    p = _to_dev(torch, inputs.gauss_mixture_1d(n, rng))
    q = _to_dev(torch, inputs.gauss_mixture_1d(n, rng))
    C = gw.grad(X, X, p, q, torch.outer(p, q))
    _, _, _, e50 = gw.sinkhorn_tol(C, p, q, eps, 50, every, -1.0, c_scale=2.0)
    tol = 0.5 * float(e50.item())
    f, g, done, e = gw.sinkhorn_tol(C, p, q, eps, cap, every, tol, c_scale=2.0)
    torch.cuda.synchronize()
    k = int(done.item())
    print(f"n=4096 tol {tol:.3e} met after {k} iterations, err {float(e.item()):.3e}", flush=True)
    assert k % every == 0 and 2 * every <= k < cap
    assert float(e.item()) <= tol
    f2, g2 = gw.sinkhorn(C, p, q, eps, k, c_scale=2.0)
    assert torch.equal(f, f2) and torch.equal(g, g2)
    _, _, done3, e3 = gw.sinkhorn_tol(C, p, q, eps, k - every, every, tol, c_scale=2.0)
    torch.cuda.synchronize()
    assert int(done3.item()) == k - every and float(e3.item()) > tol


@pytest.mark.parametrize("sx,sy,kx,ky,eps,every,path", [((120,), (100,), 1, 2, 0.01, 5, "fast"),
                                                        ((90,), (140,), 2, 2, 0.005, 4, "dense"),
                                                        ((9, 11), (10, 10), 1, 1, 0.02, 3, "fast")])
def test_solve_tol_matches_oracle(sx, sy, kx, ky, eps, every, path):
    gw, torch = _gw()
    print(f"solve_tol {sx} {sy} eps={eps} every={every} {path}", flush=True)
    X, Y = gw.unit_grid(sx, kx), gw.unit_grid(sy, ky)
    gx, gy = ogrid(X), ogrid(Y)
    rng = inputs.rng_for(913, X.size, Y.size)
    if len(sx) == 1:
        p, q = inputs.gauss_mixture_1d(X.size, rng), inputs.gauss_mixture_1d(Y.size, rng)
    else:
        p = inputs.blobs_2d(sx[0], sx[1], rng, floor=1e-6)
        q = inputs.blobs_2d(sy[0], sy[1], rng, floor=1e-6)
    outer, max_inner = 3, 150
    # a tol that no outer step's violation trajectory comes near (ratio 1.05)
    tol = None
    for cand in (1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 3e-6, 1e-6):
        T = p[:, None] * q[None, :]
        ok = True
        for _ in range(outer):
            C = 2.0 * O.grad_dense(gx, gy, p, q, T)
            errs = _check_errs(C, p, q, eps, every, max_inner // every, below=cand)
            if any(abs(np.log(e / cand)) < np.log(1.05) for e in errs):
                ok = False
                break
            f, g, _, _ = O.sinkhorn_tol(C, p, q, eps, max_inner, every, cand)
            T = O.plan(C, f, g, eps)
        if ok:
            tol = cand
            break
    assert tol is not None
    T0, f0, g0, (E0, R0), done0 = O.solve_tol(gx, gy, p, q, eps, outer, max_inner, every, tol)
    T, f, g, obj, done = gw.solve_tol(X, Y, _to_dev(torch, p), _to_dev(torch, q), eps, outer,
                                      max_inner, every, tol, path=path)
    torch.cuda.synchronize()
    assert done.cpu().tolist() == done0
    assert err(T.cpu().numpy(), T0) <= TOL
    assert err(f.cpu().numpy(), f0) <= TOL and err(g.cpu().numpy(), g0) <= TOL
    o = obj.cpu().numpy()
    assert abs(o[0] - E0) <= TOL * abs(E0)


def test_tol_rejects_bad_arguments():
    gw, torch = _gw()
    C = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    z = torch.full((4,), 0.25, dtype=torch.float64, device="cuda")
    with pytest.raises(gw.GWError):
        gw.sinkhorn_tol(C, z, z, 0.1, 10, 0, 1e-3)
    with pytest.raises(gw.GWError):
        gw.sinkhorn_tol(C, z, z, 0.1, 10, 2, float("nan"))
    X = gw.unit_grid((4,), 1)
    with pytest.raises(gw.GWError):
        gw.solve_tol(X, X, z, z, 0.1, 1, 10, 0, 1e-3)
