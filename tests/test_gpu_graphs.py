"""Whole calls captured into HIP graphs (torch.cuda.CUDAGraph on a side
stream): the library enqueues only kernels on the caller's stream (no host
waits, no memsets, no allocations), so a captured gradient or solve replays
the eager call's arithmetic.  Each case replays three times, with eager work
of the library between the replays, and every replay must equal the eager
result bit for bit."""
import pytest

from paper_2404_08970_amd import inputs

from test_gpu_parity import _gw, _to_dev

pytestmark = pytest.mark.gpu


def _replay_equal(torch, graph, outs, refs, between):
    for r in range(3):
        print(f"replay {r}", flush=True)
        graph.replay()
        torch.cuda.synchronize()
        for o, ref in zip(outs, refs):
            assert torch.equal(o, ref)
        between()
        torch.cuda.synchronize()


@pytest.mark.parametrize("sx,sy,k,metric", [((700,), (513,), 2, 0), ((20, 24), (18, 18), 2, 1),
                                            ((9, 10), (12, 8), 2, 0), ((6, 7, 8), (300,), 1, 0)])
def test_grad_graph_replays_equal_eager(sx, sy, k, metric):
    gw, torch = _gw()
    X = gw.unit_grid(sx, k, metric)
    Y = gw.unit_grid(sy, k, metric if len(sy) > 1 else 0)
    rng = inputs.rng_for(970, X.size, Y.size)
    T = _to_dev(torch, inputs.random_plan(X.size, Y.size, rng))
    p = _to_dev(torch, inputs.dirichlet(X.size, rng))
    q = _to_dev(torch, inputs.dirichlet(Y.size, rng))
    G0 = gw.grad(X, Y, p, q, T).clone()  # eager (also sets any kernel attributes once)
    torch.cuda.synchronize()
    ws = gw.workspace(gw.workspace_bytes(X, Y, gw.PATH_FAST_F64, gw.OP_GRAD), "cuda", key="cap_g")
    G = torch.empty_like(G0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        gw.grad(X, Y, p, q, T, out=G, ws=ws)
    _replay_equal(torch, graph, [G], [G0], lambda: gw.grad(X, Y, p, q, T))


@pytest.mark.parametrize("sx,sy,k,metric,warm", [((300,), (257,), 1, 0, False),
                                                 ((16, 16), (12, 20), 2, 1, True)])
def test_solve_graph_replays_equal_eager(sx, sy, k, metric, warm):
    gw, torch = _gw()
    X = gw.unit_grid(sx, k, metric)
    Y = gw.unit_grid(sy, k, metric if len(sy) > 1 else 0)
    rng = inputs.rng_for(971, X.size, Y.size)
    p = _to_dev(torch, inputs.dirichlet(X.size, rng))
    q = _to_dev(torch, inputs.dirichlet(Y.size, rng))
    eps, outer, inner = 5e-3, 3, 20
    T0, f0, g0, o0 = (t.clone() for t in gw.solve(X, Y, p, q, eps, outer, inner, warm=warm))
    torch.cuda.synchronize()
    ws = gw.workspace(gw.workspace_bytes(X, Y, gw.PATH_FAST_F64, gw.OP_SOLVE), "cuda", key="cap_s")
    T, f, g, o = (torch.empty_like(t) for t in (T0, f0, g0, o0))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        gw.solve(X, Y, p, q, eps, outer, inner, warm=warm, T=T, f=f, g=g, obj=o, ws=ws)
    _replay_equal(torch, graph, [T, f, g, o], [T0, f0, g0, o0],
                  lambda: gw.solve(X, Y, p, q, eps, 1, 5))
