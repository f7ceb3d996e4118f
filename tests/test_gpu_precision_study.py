"""The precision study at its size: dense gradients on FP32 and BF16 matrix
cores (and their split refinements) against the FP64 oracle at n = 16384,
k = 2, Dirichlet(1) marginals, on the plans p q^T and one FAST outer step
(eps = 1e-3, 100 Sinkhorn iterations).  The oracle computes sampled rows of G
from the plain definition (grad_rows); each path's error relative to the
largest |2 D_X T D_Y| of those rows must stay within its a-priori bound (the
FP64 paths within 1e-12), and is printed."""
import numpy as np
import pytest

from oracle import gw_oracle as O
from paper_2404_08970_amd import inputs
from test_gpu_parity import lp_bound

pytestmark = pytest.mark.gpu


def _gw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_08970_amd import gw
    return gw, torch


def test_precision_study_n16384_against_oracle():
    gw, torch = _gw()
    n, k = 16384, 2
    print(f"precision study n={n} k={k}", flush=True)
    dev = torch.device("cuda")
    X = gw.unit_grid((n,), k)
    p = inputs.dirichlet(n, inputs.rng_for(4, 0))
    q = inputs.dirichlet(n, inputs.rng_for(4, 1))
    pd, qd = torch.tensor(p, device=dev), torch.tensor(q, device=dev)
    plans = {"pq": torch.outer(pd, qd)}
    plans["one_outer_step"] = gw.solve(X, X, pd, qd, 1e-3, 1, 100, path="fast", objective=False)[0]
    paths = ["fast", "dense_f64", "dense_f32", "dense_bf16", "dense_f32_split", "dense_bf16_split"]
    rows = np.linspace(0, n - 1, 6).astype(int)
    og = O.Grid((n,), X.h, k)
    for name, T in plans.items():
        Tc = T.cpu().numpy()
        ref = O.grad_rows(og, og, p, q, Tc, rows)
        del Tc
        # the constant terms alone (T = 0): the bilinear part is const - ref
        const = O.grad_rows(og, og, p, q, np.zeros((n, n)), rows)
        scale = float(np.max(np.abs(const - ref)))
        for pth in paths:
            G = gw.grad(X, X, pd, qd, T, path=pth)
            torch.cuda.synchronize()
            e = float(np.max(np.abs(G[torch.tensor(rows, device=dev)].cpu().numpy() - ref))) / scale
            del G
            bound = 1e-12 if pth in ("fast", "dense_f64") else lp_bound(pth, n)
            print(f"  {name} {pth}: err_bilinear={e:.3e} bound={bound:.3e}", flush=True)
            assert e <= bound
