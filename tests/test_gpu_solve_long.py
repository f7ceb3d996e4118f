"""GPU parity of whole solves at the iteration counts the workloads run.

* Many-outer solves (100 mirror-descent steps x 100 Sinkhorn iterations) on
  1D grids (n = 384, k = 1, 2, 3; FAST and dense gradients) and on a 32 x 32
  squared-Euclidean 2D grid; the 64 x 64 2D workload's first two outer steps;
  an (l1)^k 2D solve with image sides above 64 (the generic grid operator).
  Expected values are the CPU oracle's, written by
  tests/golden/make_solve_fixtures.py (which calls only the oracle): the final
  potentials, the objective, the plan's row and column sums and sampled rows
  of the plan, compared element by element.
* The 1D uniform-marginal workload: n = 200 on [0, 1], |x_i - x_j|^2,
  p = q uniform, eps = 5e-3, 50 outer x 100 Sinkhorn iterations, dense FP64
  gradient (and FAST), against the oracle computed here.  GW is invariant
  under reflecting a grid (Sec. 1, the invariances of the GW distance), the
  start p q^T is reflection-symmetric and rounding decides which of the two
  mirror-image optima the iteration approaches, so the plan must equal the
  oracle's T or its reflection R_X T (rows reversed), whichever is closer,
  with the potentials reflected alike; the objective must match either way.

Tolerance: relative 1e-10 (FP64 paths)."""
import json
import os

import numpy as np
import pytest

from oracle import gw_oracle as O
from paper_2404_08970_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _gw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_08970_amd import gw
    return gw, torch


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _rel(x, ref):
    x, ref = np.asarray(x, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(x)), "non-finite pattern differs"
    if not fin.any():
        return 0.0
    return float(np.max(np.abs(x[fin] - ref[fin])) / np.max(np.abs(ref[fin])))


def _load(name):
    z = np.load(os.path.join(GOLDEN, f"solve_{name}.npz"), allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    return z, meta


def _marginal(meta, shape, side):
    rng = inputs.rng_for(*meta["key"], side)
    if meta["marg"] == "mix":
        return inputs.gauss_mixture_1d(shape[0], rng)
    return inputs.blobs_2d(shape[0], shape[1], rng, floor=meta.get("floor", 0.0))


FIXTURE_RUNS = [("1d_n384_k1", "fast"), ("1d_n384_k1", "dense"),
                ("1d_n384_k2", "fast"), ("1d_n384_k2", "dense"),
                ("1d_n384_k3", "fast"), ("1d_n384_k3", "dense"),
                ("2d_32x32_sqeuclid", "fast"), ("2d_64x64_sqeuclid", "fast"),
                ("2d_70x66_k2_65x80_k3", "fast")]


@pytest.mark.parametrize("name,path", FIXTURE_RUNS)
def test_long_solve_matches_oracle_fixture(name, path):
    gw, torch = _gw()
    z, meta = _load(name)
    print(f"long solve {name} {path} {meta['outer']}x{meta['inner']}", flush=True)
    (sx, kx, mx), (sy, ky, my) = meta["X"], meta["Y"]
    X = gw.Grid(tuple(sx), meta["hx"], kx, mx)
    Y = gw.Grid(tuple(sy), meta["hy"], ky, my)
    p, q = _marginal(meta, sx, 0), _marginal(meta, sy, 1)
    T, f, g, obj = gw.solve(X, Y, _dev(torch, p), _dev(torch, q), meta["eps"], meta["outer"],
                            meta["inner"], path=path)
    torch.cuda.synchronize()
    gw.check_status()
    rows = z["rows"]
    Tn = T.cpu().numpy()
    o = obj.cpu().numpy()
    errs = {"f": _rel(f.cpu().numpy(), z["f"]), "g": _rel(g.cpu().numpy(), z["g"]),
            "rowsum": _rel(Tn.sum(axis=1), z["rowsum"]), "colsum": _rel(Tn.sum(axis=0), z["colsum"]),
            "T_rows": _rel(Tn[rows], z["T_rows"]),
            "E": abs(o[0] - z["obj"][0]) / abs(z["obj"][0]),
            "E+epsH": abs(o[1] - z["obj"][1]) / max(abs(z["obj"][1]), abs(z["obj"][0]))}
    print("  " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    for k, v in errs.items():
        assert v <= TOL, (k, v)


def _config1():
    n, k, eps, outer, inner = 200, 2, 5e-3, 50, 100
    p = np.full(n, 1.0 / n)
    return n, k, eps, outer, inner, p


_CONFIG1_ORACLE = {}


def _config1_oracle():
    if "r" not in _CONFIG1_ORACLE:
        n, k, eps, outer, inner, p = _config1()
        og = O.Grid((n,), 1.0 / (n - 1), k)
        _CONFIG1_ORACLE["r"] = O.solve(og, og, p, p, eps, outer, inner)
    return _CONFIG1_ORACLE["r"]


@pytest.mark.parametrize("path", ["dense", "fast"])
def test_uniform_1d_n200_workload_up_to_reflection(path):
    gw, torch = _gw()
    n, k, eps, outer, inner, p = _config1()
    print(f"uniform 1D n={n} k={k} eps={eps} {outer}x{inner} {path}", flush=True)
    X = gw.unit_grid((n,), k)
    pd = _dev(torch, p)
    T, f, g, obj = gw.solve(X, X, pd, pd, eps, outer, inner, path=path)
    torch.cuda.synchronize()
    gw.check_status()
    T0, f0, g0, (E0, R0) = _config1_oracle()
    Tn, fn, gn, o = T.cpu().numpy(), f.cpu().numpy(), g.cpu().numpy(), obj.cpu().numpy()
    # the two mirror images: identity on X, or rows reversed (R_X T, R_X f); g is
    # the potential of Y and stays as it is
    cands = {"T": (T0, f0, g0), "R_X T": (T0[::-1], f0[::-1], g0)}
    d = {name: _rel(Tn, c[0]) for name, c in cands.items()}
    pick = min(d, key=d.get)
    Tr, fr, gr = cands[pick]
    e_T, e_f, e_g = _rel(Tn, Tr), _rel(fn, fr), _rel(gn, gr)
    asym = float(np.max(np.abs(T0 - T0[::-1])) / np.max(T0))
    print(f"  matched {pick}: T {e_T:.2e} f {e_f:.2e} g {e_g:.2e} E {abs(o[0]-E0)/abs(E0):.2e}; "
          f"oracle plan asymmetry max|T - R_X T|/max T = {asym:.2e}", flush=True)
    assert abs(o[0] - E0) <= TOL * abs(E0)
    assert abs(o[1] - R0) <= TOL * max(abs(R0), abs(E0))
    assert e_T <= TOL and e_f <= TOL and e_g <= TOL
