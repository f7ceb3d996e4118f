"""GPU tests of the request loop through the C ABI.

A request's result must be the same bits as gw_solve on the FAST path with the
same arguments (each band of each iteration runs the single-problem kernel's
arithmetic and no reduction crosses requests), whether the request runs alone
or in a mix; one small case is also checked against the CPU oracle
(relative error <= 1e-10)."""
import numpy as np
import pytest

from oracle import gw_oracle as O
from paper_2404_08970_amd import inputs

pytestmark = pytest.mark.gpu

GB = 1 << 30


def _gw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_08970_amd import gw
    return gw, torch


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _case(gw, torch, seed, xshape, yshape, k, metric=0, ky=None):
    rng = inputs.rng_for(500, seed)
    X = gw.unit_grid(xshape, k, metric)
    Y = gw.unit_grid(yshape, ky if ky is not None else k, metric)

    def marg(shape):
        if len(shape) == 1:
            return inputs.gauss_mixture_1d(shape[0], rng)
        if len(shape) == 2:
            return inputs.blobs_2d(shape[0], shape[1], rng)
        return inputs.blobs_3d(*shape, rng, floor=1e-6)
    return X, Y, _dev(torch, marg(xshape)), _dev(torch, marg(yshape))


def _reference(gw, torch, X, Y, p, q, eps, outer, inner, warm, objective):
    T, f, g, obj = gw.solve(X, Y, p, q, eps, outer, inner, path="fast", warm=warm,
                            objective=objective)
    torch.cuda.synchronize()
    return {"T": T.clone(), "f": f.clone(), "g": g.clone(),
            "obj": tuple(obj.cpu().tolist()) if objective else None}


def _run_until_done(sv, ids, max_steps=100000):
    done = {}
    for _ in range(max_steps):
        sv.step()
        for rid in ids:
            if rid not in done and sv.poll(rid) == 2:
                done[rid] = sv.result(rid)
        if len(done) == len(ids):
            return done
    raise AssertionError("requests did not finish")


def _assert_same(torch, res, ref, objective):
    assert res["status"] == 0
    assert torch.equal(res["T"], ref["T"])
    assert torch.equal(res["f"], ref["f"])
    assert torch.equal(res["g"], ref["g"])
    if objective:
        assert res["obj"] == ref["obj"]


# (xshape, yshape, k, metric, eps, outer, inner, warm, objective): one case per
# row-pass length class, a 2D grid, and a 1D x 2D pair with M != N
CLASS_CASES = [
    ((100,), (100,), 1, 0, 5e-3, 2, 7, False, True),
    ((300,), (300,), 2, 0, 2e-3, 2, 7, True, False),
    ((700,), (700,), 2, 0, 1e-2, 2, 7, False, False),
    ((1500,), (1500,), 1, 0, 3e-3, 2, 7, True, True),
    ((3000,), (3000,), 2, 0, 1e-3, 2, 7, False, False),
    ((5000,), (5000,), 1, 0, 4e-3, 2, 7, False, True),
    ((100, 100), (100, 100), 1, 0, 5e-3, 1, 4, False, False),
    ((257,), (12, 12), 2, 1, 2e-3, 3, 5, True, True),
    ((2500,), (2500,), 1, 0, 3e-3, 1, 5, False, False),
    ((96, 96), (96, 96), 2, 0, 4e-3, 1, 4, True, True),
    ((128, 128), (128, 128), 1, 0, 6e-3, 1, 3, False, False),
    ((12, 12, 12), (10, 10, 10), 2, 1, 3e-3, 2, 5, False, True),  # 3D, axis-separable
    ((8, 8, 8), (7, 9, 6), 2, 0, 5e-3, 2, 4, True, True),         # 3D (l1)^2, 3D image operator
    ((40, 50), (64, 64), 2, 0, 4e-3, 2, 4, False, True),          # 2D (l1)^2, image operator
]


@pytest.mark.parametrize("xs,ys,k,metric,eps,outer,inner,warm,objective", CLASS_CASES)
def test_alone_equals_solve(xs, ys, k, metric, eps, outer, inner, warm, objective):
    gw, torch = _gw()
    X, Y, p, q = _case(gw, torch, len(xs) * 10000 + xs[0], xs, ys, k, metric)
    print(f"serve alone {xs}x{ys} k={k} metric={metric} outer={outer} inner={inner}", flush=True)
    ref = _reference(gw, torch, X, Y, p, q, eps, outer, inner, warm, objective)
    sv = gw.Server(gw.request_bytes(X, Y) + gw.server_table_bytes(2) + (1 << 20), max_slots=2,
                   iters_per_step=3)
    rid = sv.submit(X, Y, p, q, eps, outer, inner, warm=warm, objective=objective)
    res = _run_until_done(sv, [rid])[rid]
    _assert_same(torch, res, ref, objective)
    sv.release(rid)
    sv.close()


def test_mix_equals_alone():
    """Staggered submissions of uneven sizes with fewer slots than requests:
    every result equals its standalone solve bit for bit.  (inner = 0 is run
    with one outer step only: without Sinkhorn the plan's mass is not 1 and a
    second gradient overflows, in gw_solve as here.)"""
    gw, torch = _gw()
    specs = [((128,), 1, 0, 5e-3, 2, 9, False, True), ((2000,), 2, 0, 2e-3, 2, 9, True, False),
             ((513,), 1, 0, 1e-2, 3, 4, False, True), ((40, 40), 1, 0, 3e-3, 2, 9, False, False),
             ((4000,), 1, 0, 1e-3, 1, 9, False, True), ((96, 96), 2, 0, 6e-3, 1, 5, True, False),
             ((1024,), 2, 0, 2e-3, 1, 0, False, True), ((6000,), 2, 0, 7e-3, 1, 3, False, False),
             ((300,), 1, 0, 4e-3, 0, 5, False, True), ((777,), 1, 0, 5e-3, 2, 11, True, True)]
    cases = []
    for i, (shape, k, metric, eps, outer, inner, warm, obj) in enumerate(specs):
        X, Y, p, q = _case(gw, torch, 900 + i, shape, shape, k, metric)
        cases.append((X, Y, p, q, eps, outer, inner, warm, obj))
    refs = []
    for X, Y, p, q, eps, outer, inner, warm, obj in cases:
        if outer == 0:
            refs.append(None)
            continue
        refs.append(_reference(gw, torch, X, Y, p, q, eps, outer, inner, warm, obj))
    sv = gw.Server(6 * GB, max_slots=4, iters_per_step=4)
    ids = []
    schedule = [3, 0, 0, 3, 0, 2, 0, 0, 2]  # submissions before each of the first steps
    it = iter(cases)
    for n_sub in schedule:
        for _ in range(n_sub):
            X, Y, p, q, eps, outer, inner, warm, obj = next(it)
            ids.append(sv.submit(X, Y, p, q, eps, outer, inner, warm=warm, objective=obj))
        sv.step()
    assert len(ids) == len(cases)
    done = _run_until_done(sv, ids)
    for rid, ref, c in zip(ids, refs, cases):
        res = done[rid]
        print(f"mix request {rid} shape={c[0].shape} outer={c[5]} inner={c[6]}", flush=True)
        if ref is None:  # outer = 0: T = p q^T
            X, Y, p, q = c[:4]
            assert torch.equal(res["T"], torch.outer(p, q))
            continue
        _assert_same(torch, res, ref, c[8])
    # the same requests alone give the same bits as in the mix (spot check)
    for j in (1, 3, 9):
        X, Y, p, q, eps, outer, inner, warm, obj = cases[j]
        sv2 = gw.Server(2 * GB, max_slots=1, iters_per_step=7)
        r2 = sv2.submit(X, Y, p, q, eps, outer, inner, warm=warm, objective=obj)
        alone = _run_until_done(sv2, [r2])[r2]
        assert torch.equal(alone["T"], done[ids[j]]["T"])
        assert torch.equal(alone["g"], done[ids[j]]["g"])
        sv2.close()
    for rid in ids:
        sv.release(rid)
    sv.close()


def test_size_quotas_keep_results():
    """Size quotas (boost 8, 3 iterations per step): requests with at most
    1/2, 1/4, 1/8 of the largest problem take 6, 12, 24 iterations a step,
    calls whose remainder is below the quota take the remainder; every result
    is still gw_solve's bits, and the smallest request needs fewer steps than
    the largest."""
    gw, torch = _gw()
    specs = [((4000,), 1, 2e-3, 2, 23, False, True), ((128,), 2, 5e-3, 3, 23, True, True),
             ((30, 30), 1, 4e-3, 2, 17, False, False), ((1000,), 2, 3e-3, 2, 23, False, True),
             ((2000,), 1, 6e-3, 1, 9, True, False), ((2900,), 2, 2e-3, 1, 14, False, False)]
    cases, refs = [], []
    for i, (shape, k, eps, outer, inner, warm, obj) in enumerate(specs):
        X, Y, p, q = _case(gw, torch, 950 + i, shape, shape, k)
        cases.append((X, Y, p, q, eps, outer, inner, warm, obj))
        refs.append(_reference(gw, torch, X, Y, p, q, eps, outer, inner, warm, obj))
    sv = gw.Server(6 * GB, max_slots=8, iters_per_step=3, boost=8)
    ids = [sv.submit(X, Y, p, q, eps, outer, inner, warm=warm, objective=obj)
           for X, Y, p, q, eps, outer, inner, warm, obj in cases]
    finished = {}
    for n in range(1, 10000):
        sv.step()
        for rid in ids:
            if rid not in finished and sv.poll(rid) == 2:
                finished[rid] = n
        if len(finished) == len(ids):
            break
    for rid, ref, c in zip(ids, refs, cases):
        print(f"quota request {rid} shape={c[0].shape} finished at step {finished[rid]}", flush=True)
        _assert_same(torch, sv.result(rid), ref, c[8])
    assert finished[ids[1]] < finished[ids[0]]
    for b in (0, 3, 16, -2):
        with pytest.raises(gw.GWError):
            sv.set_boost(b)
    sv.set_boost(1)
    for rid in ids:
        sv.release(rid)
    sv.close()
    sv2 = gw.Server(gw.server_table_bytes(1) + 4096, max_slots=1, iters_per_step=200)
    sv2.set_boost(4)
    with pytest.raises(gw.GWError):
        sv2.set_boost(8)       # 200 x 8 iterations exceed a step's 1000
    sv2.close()


def test_graph_cache_eviction_keeps_results():
    """More distinct step graphs than the server keeps (256): each step runs a
    different set of row-length classes (pairs, triples and quadruples of the
    11 classes, one 2 x N request per class), so the least recently used
    graphs are destroyed and, when a class set comes back, captured again.
    Every result equals the request's gw_solve bit for bit."""
    import itertools
    gw, torch = _gw()
    Ns = [200, 400, 900, 1800, 2900, 3900, 5000, 7000, 9000, 11000, 15000]  # one per class
    X = gw.unit_grid((2,), 1)
    p = torch.tensor([0.3, 0.7], dtype=torch.float64, device="cuda")
    rng = inputs.rng_for(960)
    cls = []
    for n in Ns:
        Y = gw.unit_grid((n,), 2)
        q = _dev(torch, inputs.gauss_mixture_1d(n, rng))
        cls.append((Y, q, _reference(gw, torch, X, Y, p, q, 4e-3, 1, 3, False, False)))
    subsets = (list(itertools.combinations(range(11), 2)) +
               list(itertools.combinations(range(11), 3)) +
               list(itertools.combinations(range(11), 4))[:60])
    assert len(subsets) > 256
    sv = gw.Server(GB, max_slots=8, iters_per_step=3)
    for n_set, sub in enumerate(subsets + subsets[:5]):  # the first sets again, after eviction
        ids = [sv.submit(X, cls[c][0], p, cls[c][1], 4e-3, 1, 3) for c in sub]
        done = _run_until_done(sv, ids)
        for rid, c in zip(ids, sub):
            _assert_same(torch, done[rid], cls[c][2], False)
            sv.release(rid)
        if n_set % 50 == 0:
            print(f"class set {n_set}: {sub}", flush=True)
    sv.close()


def test_admission_by_footprint():
    gw, torch = _gw()
    X, Y, p, q = _case(gw, torch, 31, (1000,), (1000,), 2)
    fp = gw.request_bytes(X, Y)
    sv = gw.Server(gw.server_table_bytes(4) + 2 * fp + 4096, max_slots=4, iters_per_step=5)
    ids = [sv.submit(X, Y, p, q, 3e-3, 2, 10) for _ in range(3)]
    sv.step()
    states = [sv.poll(r) for r in ids]
    assert states[2] == 0 and states[0] != 0 and states[1] != 0   # memory admits two
    assert sv.result(ids[0]) is None                               # not finished
    with pytest.raises(gw.GWError) as ei:
        sv.release(ids[0])
    assert ei.value.status == gw.GW_EAGAIN
    for _ in range(200):
        sv.step()
        if sv.poll(ids[0]) == 2 and sv.poll(ids[1]) == 2:
            break
    assert sv.poll(ids[0]) == 2 and sv.poll(ids[1]) == 2
    sv.step()
    assert sv.poll(ids[2]) == 0            # finished requests keep their memory
    sv.release(ids[0])
    sv.step()
    assert sv.poll(ids[2]) != 0            # admitted once a range is free
    done = _run_until_done(sv, [ids[2]])
    ref = _reference(gw, torch, X, Y, p, q, 3e-3, 2, 10, False, False)
    _assert_same(torch, done[ids[2]], ref, False)
    a = sv.result(ids[1])
    _assert_same(torch, a, ref, False)     # identical inputs, identical bits
    sv.release(ids[1]); sv.release(ids[2])
    sv.close()


def test_errors():
    gw, torch = _gw()
    X, Y, p, q = _case(gw, torch, 41, (200,), (200,), 1)
    sv = gw.Server(gw.server_table_bytes(2) + gw.request_bytes(X, Y) + 4096, max_slots=2)
    big = gw.unit_grid((600,), 1)
    pb = torch.full((600,), 1 / 600, dtype=torch.float64, device="cuda")
    with pytest.raises(gw.GWError) as ei:
        sv.submit(big, big, pb, pb, 1e-2, 1, 1)          # footprint above the arena
    assert ei.value.status == gw.GW_ENOMEM
    wide = gw.unit_grid((16385,), 1)
    pw = torch.full((16385,), 1 / 16385, dtype=torch.float64, device="cuda")
    with pytest.raises(gw.GWError) as ei:
        sv.submit(X, wide, p, pw, 1e-2, 1, 1)
    assert ei.value.status == gw.GW_EUNSUPPORTED
    with pytest.raises(gw.GWError) as ei:
        sv.poll(12345)
    assert ei.value.status == gw.GW_EINVAL
    rid = sv.submit(X, Y, p, q, 1e-2, 1, 3)
    assert sv.poll(rid) == 0
    sv.release(rid)                                        # a queued request can be dropped
    with pytest.raises(gw.GWError):
        sv.poll(rid)
    sv.close()


def test_small_request_matches_oracle():
    gw, torch = _gw()
    n, k, eps, outer, inner = 48, 2, 1e-2, 3, 20
    X, Y, p, q = _case(gw, torch, 51, (n,), (n,), k)
    sv = gw.Server(GB // 4, max_slots=2, iters_per_step=6)
    rid = sv.submit(X, Y, p, q, eps, outer, inner, objective=True)
    res = _run_until_done(sv, [rid])[rid]
    og = O.Grid((n,), X.h, k)
    T0, f0, g0, obj0 = O.solve(og, og, p.cpu().numpy(), q.cpu().numpy(), eps, outer, inner)
    T = res["T"].cpu().numpy()
    assert np.max(np.abs(T - T0)) <= 1e-10 * np.max(np.abs(T0))
    assert abs(res["obj"][0] - obj0[0]) <= 1e-10 * abs(obj0[0])
    sv.release(rid)
    sv.close()
