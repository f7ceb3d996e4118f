"""Plain FP64 CPU oracle for entropic Gromov-Wasserstein on uniform grids.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The product path (the
HIP library and its Python binding) never calls it, and it shares no code with
that path: no kernels, tables, helpers or pre/post-processing.

Everything here is written to be read against the paper (arXiv 2404.08970,
"Fast Gradient Computation for Gromov-Wasserstein Distance"):

* grids and cost matrices ........ Sec. 2, Eq. (1d distance matrices);
                                   Sec. 3.1, Eq. (2d Dx) and the D_1 / J display
* QAP objective .................. Sec. 2, discrete GW objective E(Gamma)
* entropic GW, entropy H ......... Sec. 2, Eq. (entropic GW)
* gradient decomposition ......... Sec. 2, C_1 - 4 D_X Gamma D_Y (after
                                   Eq. gradient entry); the value returned
                                   here is G = grad E / 2
* mirror descent with tau = eps .. Sec. 2.1, Eq. (GW sinkhorn) and the
                                   Remark on tau = eps
* Sinkhorn ....................... cited by the paper (Cuturi 2013); written
                                   here in log domain (readings below), with an
                                   optional tolerance stop
* Pascal recursion for L x ....... Sec. 3, Eq. (1d y), Eq. (1d recursive relation)
* four-term split of D Gamma D ... Sec. 3, Eq. (Dx)
* 2D Kronecker expansion ......... Sec. 3.1, Eq. (2D kronecker), Eq. (2d gradient)
* 3D grids ....................... Sec. 3.1's expansion with a third factor (the
                                   section states higher dimensions work alike)
* fused GW (FGW) ................. Remark (Entropic algorithm for FGW): objective
                                   and gradient decomposition C_2 - 4 theta D Gamma D
* unbalanced GW (UGW) ............ Remark (Entropic algorithm for UGW): divergence and
                                   sub-problem; its scalar term, its unbalanced
                                   Sinkhorn and the mass rescaling follow the cited
                                   UGW work (readings in that section)

Two gradient routines are given.  ``grad_dense`` is the plain definition
G = c1 1^T + 1 c2^T - 2 D_X T D_Y with explicit distance matrices (the
"original" O(N^3) computation).  ``grad_pascal`` is the paper's exact O(N^2)
method: the recursion applied along rows, then along columns, in index order.
Both are exact rewrites of one another; the tests pin each of them against
independent facts (brute-force four-index sums, exact integer arithmetic,
closed forms, the paper's printed matrices).

Readings where the paper is silent or garbled:

* G is half of the paper's gradient; the Sinkhorn cost in a solve is 2G.
* the second constant term uses (D_Y o D_Y) q broadcast along rows.
* 0^0 = 1 in the 2D expansion (D_1^{o0} = J, diagonal included).
* D_1 = [|i-j|] (the printed last row drops its trailing 0).
* flattening of 2D grids is row-major, flat = r * W + c.
* T^0 = p q^T; Sinkhorn updates f then g, cold start each outer iteration,
  fixed iteration counts; LSE is max-shifted; p_i = 0 gives f_i = -inf.
* SQEUCLID (h^2 (dr^2 + dc^2)) is supported beside the paper's (l1)^k metric.
* 3D grids: (|dd|+|dr|+|dc|)^k or squared Euclidean, flattened row-major
  (flat = (d * H + r) * W + c).
* FGW feature cost c_ip = fa_i - fb_p (its square enters): every FGW workload
  of the paper has this form (|i - p|, signal-strength and gray-level
  differences).
* optional tolerance stop (the paper fixes iteration counts): every
  check_every iterations the column-marginal L1 violation of the half-step
  plan (f_t, g_{t-1}) is measured; the iteration completes and the loop stops
  once it is <= tol.

Precision: float64 everywhere; no fused multiply-add is requested; sums run in
index order except where a library primitive (numpy matmul / sum) is used as
one step of a plain definition.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

METRIC_L1POW = 0
METRIC_SQEUCLID = 1


@dataclass(frozen=True)
class Grid:
    """A uniform grid: 1D with ``shape=(n,)``, 2D with ``shape=(H, W)`` or 3D
    with ``shape=(D, H, W)`` (the extension of Sec. 3.1 to one more axis).

    ``h`` is the spacing, ``k`` the exponent of the distance (Sec. 2 and
    Sec. 3.1) and ``metric`` selects the l1 distance to the power k,
    (|dr|+|dc|)^k in 2D (the paper's metric) and (|dd|+|dr|+|dc|)^k in 3D, or
    the squared Euclidean distance (k must be 2)."""

    shape: tuple
    h: float
    k: int
    metric: int = METRIC_L1POW

    @property
    def ndim(self) -> int:
        return len(self.shape)

    @property
    def size(self) -> int:
        n = 1
        for s in self.shape:
            n *= int(s)
        return n


def h_power(g: Grid) -> float:
    """h^k as k left-to-right multiplications (h^2 for SQEUCLID)."""
    kk = 2 if g.metric == METRIC_SQEUCLID else g.k
    v = 1.0
    for _ in range(kk):
        v = v * g.h
    return v


def _axis_coords(g: Grid, flat) -> list:
    """Row-major coordinates of flat indices, one array per axis."""
    coords, rest = [], np.asarray(flat, dtype=np.int64)
    for ext in reversed(g.shape):
        coords.append(rest % ext)
        rest = rest // ext
    return coords[::-1]


def _distance_from_axes(g: Grid, diffs) -> np.ndarray:
    if g.metric == METRIC_SQEUCLID:
        return sum(d * d for d in diffs)
    return sum(diffs) ** g.k


def integer_distance(g: Grid) -> np.ndarray:
    """Unscaled integer distance matrix (int64), Eq. (1d distance matrices) /
    Eq. (2d Dx) and its 3D analogue.  Multi-dimensional grids are flattened
    row-major."""
    if g.ndim == 1:
        idx = np.arange(g.shape[0], dtype=np.int64)
        d = np.abs(idx[:, None] - idx[None, :])
        return d ** g.k
    if g.ndim == 3:
        co = _axis_coords(g, np.arange(g.size))
        return _distance_from_axes(g, [np.abs(c[:, None] - c[None, :]) for c in co])
    H, W = g.shape
    flat = np.arange(H * W, dtype=np.int64)
    r, c = flat // W, flat % W
    dr = np.abs(r[:, None] - r[None, :])
    dc = np.abs(c[:, None] - c[None, :])
    if g.metric == METRIC_SQEUCLID:
        return dr * dr + dc * dc
    return (dr + dc) ** g.k


def cost_matrix(g: Grid) -> np.ndarray:
    """D = h^k * (integer distance), float64 (exact integers below 2^53)."""
    return h_power(g) * integer_distance(g).astype(np.float64)


def integer_distance_rows(g: Grid, rows) -> np.ndarray:
    """Rows `rows` of integer_distance(g), by the same definition, for grids too
    large to form the whole matrix."""
    rows = np.asarray(rows, dtype=np.int64)
    if g.ndim == 1:
        idx = np.arange(g.shape[0], dtype=np.int64)
        return np.abs(rows[:, None] - idx[None, :]) ** g.k
    if g.ndim == 3:
        ca, cb = _axis_coords(g, rows), _axis_coords(g, np.arange(g.size))
        return _distance_from_axes(g, [np.abs(a[:, None] - b[None, :]) for a, b in zip(ca, cb)])
    H, W = g.shape
    flat = np.arange(H * W, dtype=np.int64)
    r, c = flat // W, flat % W
    dr = np.abs((rows // W)[:, None] - r[None, :])
    dc = np.abs((rows % W)[:, None] - c[None, :])
    if g.metric == METRIC_SQEUCLID:
        return dr * dr + dc * dc
    return (dr + dc) ** g.k


# ---------------------------------------------------------------------------
# Gradient: plain definition (the "original" computation)
# ---------------------------------------------------------------------------

def const_terms(DX: np.ndarray, DY: np.ndarray, p: np.ndarray, q: np.ndarray):
    """c1 = (D_X o D_X) p and c2 = (D_Y o D_Y) q (Sec. 2, constant term C_1)."""
    return (DX * DX) @ p, (DY * DY) @ q


def grad_dense(gx: Grid, gy: Grid, p, q, T) -> np.ndarray:
    """G = c1 1^T + 1 c2^T - 2 D_X T D_Y  (= half the paper's gradient)."""
    DX, DY = cost_matrix(gx), cost_matrix(gy)
    c1, c2 = const_terms(DX, DY, p, q)
    return c1[:, None] + c2[None, :] - 2.0 * ((DX @ T) @ DY)


# ---------------------------------------------------------------------------
# Gradient: the paper's recursion (Sec. 3)
# ---------------------------------------------------------------------------

def grad_rows(gx: Grid, gy: Grid, p, q, T, rows, block: int = 1024) -> np.ndarray:
    """Rows `rows` of grad_dense(gx, gy, p, q, T) by the same plain definition,
    G[rows] = c1[rows] 1^T + 1 c2^T - 2 D_X[rows] T D_Y (Sec. 2), with D_Y and
    c2 = (D_Y o D_Y) q taken in blocks of rows of D_Y so that grids of 16384
    points need no N x N distance matrix.  D_Y is symmetric, so its row blocks
    are also its column blocks."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    DXr = h_power(gx) * integer_distance_rows(gx, rows).astype(np.float64)
    c1r = (DXr * DXr) @ p
    Wr = DXr @ T
    N = gy.size
    acc = np.zeros((rows.shape[0], N))
    c2 = np.zeros(N)
    hy = h_power(gy)
    for j0 in range(0, N, block):
        j1 = min(N, j0 + block)
        DYb = hy * integer_distance_rows(gy, np.arange(j0, j1)).astype(np.float64)
        acc += Wr[:, j0:j1] @ DYb
        c2 += (DYb * DYb).T @ q[j0:j1]
    return c1r[:, None] + c2[None, :] - 2.0 * acc


def _binomials(m: int):
    return [[math.comb(r, s) for s in range(r + 1)] for r in range(m + 1)]


def lower_apply(x: np.ndarray, m: int) -> np.ndarray:
    """y = L x along axis 0 of ``x`` with L_ij = (i-j)^m for i > j, else 0.

    The paper's state a_{i,r} = sum_{j<i} (i-j)^{r-1} x_j (here indexed
    r = 0..m) starts at zero and advances by
    a_{i+1,r} = x_i + sum_{s<=r} C(r,s) a_{i,s}; the output is a_{i,m}.
    Eq. (1d y) and Eq. (1d recursive relation).  Axis 0 is the recursion axis;
    any further axes are independent lines processed together."""
    n = x.shape[0]
    B = _binomials(m)
    a = [np.zeros(x.shape[1:], dtype=np.float64) for _ in range(m + 1)]
    y = np.empty_like(x, dtype=np.float64)
    for i in range(n):
        y[i] = a[m]
        new = []
        for r in range(m + 1):
            acc = np.array(x[i], dtype=np.float64, copy=True)
            for s in range(r + 1):
                acc = acc + B[r][s] * a[s]
            new.append(acc)
        a = new
    return y


def upper_apply(x: np.ndarray, m: int) -> np.ndarray:
    """y = L^T x along axis 0: the same recursion run from the last index
    backwards ("L^T x can be computed in a similar way", Sec. 3)."""
    return lower_apply(x[::-1], m)[::-1]


def toeplitz_apply(x: np.ndarray, m: int) -> np.ndarray:
    """[|i-j|^m] x along axis 0.  For m >= 1 this is (L + L^T) x, Eq. (Dx);
    for m = 0 it is J x (0^0 = 1, the 2D expansion's convention)."""
    if m == 0:
        total = np.sum(x, axis=0)
        return np.broadcast_to(total, x.shape).astype(np.float64)
    return lower_apply(x, m) + upper_apply(x, m)


def grid_apply(g: Grid, X: np.ndarray) -> np.ndarray:
    """Unscaled grid operator applied along axis 0 of ``X`` (shape
    (g.size, L)): 1D, [|i-j|^k]; 2D (l1)^k via Eq. (2D kronecker)
    sum_r C(k,r) D_1^{o(k-r)} mat(x) D_1^{o r}; 2D SQEUCLID via
    D^{o2} mat(x) J + J mat(x) D^{o2}."""
    if g.ndim == 1:
        return toeplitz_apply(X, g.k)
    if g.ndim == 3:
        return _grid_apply_3d(g, X)
    H, W = g.shape
    L = X.shape[1]
    img = X.reshape(H, W, L)
    out = np.zeros((H, W, L), dtype=np.float64)
    if g.metric == METRIC_SQEUCLID:
        terms = [(1, 2, 0), (1, 0, 2)]          # (coef, exponent on rows, on cols)
    else:
        terms = [(math.comb(g.k, r), g.k - r, r) for r in range(g.k + 1)]
    for coef, mr, mc in terms:
        # columns of the image (index c) first: mat(x) D^{o mc}
        t = np.transpose(img, (1, 0, 2))         # (W, H, L)
        t = toeplitz_apply(t, mc)
        t = np.transpose(t, (1, 0, 2))           # (H, W, L)
        # rows of the image (index r): D^{o mr} (...)
        t = toeplitz_apply(t, mr)
        out = out + coef * t
    return out.reshape(H * W, L)


def _grid_apply_3d(g: Grid, X: np.ndarray) -> np.ndarray:
    """3D: the Kronecker expansion of Sec. 3.1 with three factors.  (l1)^k:
    (d1 + d2 + d3)^k = sum over a + b + c = k of k!/(a! b! c!) d1^a d2^b d3^c,
    so D = sum k!/(a! b! c!) D_1^{oa} (x) D_1^{ob} (x) D_1^{oc} (D_1^{o0} = J);
    SQEUCLID: D_1^{o2} (x) J (x) J + J (x) D_1^{o2} (x) J + J (x) J (x) D_1^{o2}.
    Each factor acts along its own axis of the reshaped vector."""
    D0, H, W = g.shape
    L = X.shape[1]
    img = X.reshape(D0, H, W, L)
    if g.metric == METRIC_SQEUCLID:
        terms = [(1, (2, 0, 0)), (1, (0, 2, 0)), (1, (0, 0, 2))]
    else:
        k = g.k
        terms = [(math.factorial(k) // (math.factorial(a) * math.factorial(b) *
                                        math.factorial(k - a - b)), (a, b, k - a - b))
                 for a in range(k + 1) for b in range(k + 1 - a)]
    out = np.zeros(img.shape, dtype=np.float64)
    for coef, ms in terms:
        t = img
        for axis in (2, 1, 0):
            t = np.moveaxis(toeplitz_apply(np.moveaxis(t, axis, 0), ms[axis]), 0, axis)
        out = out + coef * t
    return out.reshape(D0 * H * W, L)


def grad_pascal(gx: Grid, gy: Grid, p, q, T) -> np.ndarray:
    """G by the paper's O(MN) method: A = T D_Y row by row, B = D_X A column
    by column, both with the recursion (Eq. (Dx), Eq. (2d gradient)); the
    constant terms use the recursion with exponent 2k (1D) or the explicit
    squared distances (2D), computed once (Sec. 2)."""
    T = np.asarray(T, dtype=np.float64)
    A = grid_apply(gy, np.ascontiguousarray(T.T)).T     # rows of T, operator on Y
    B = grid_apply(gx, np.ascontiguousarray(A))          # columns of A, operator on X
    c1 = _const_term(gx, p)
    c2 = _const_term(gy, q)
    s = h_power(gx) * h_power(gy)
    return c1[:, None] + c2[None, :] - 2.0 * (s * B)


def _const_term(g: Grid, w) -> np.ndarray:
    w = np.asarray(w, dtype=np.float64)
    if g.ndim == 1:
        hk = h_power(g)
        return (hk * hk) * toeplitz_apply(w[:, None], 2 * g.k)[:, 0]
    D = cost_matrix(g)
    return (D * D) @ w


# ---------------------------------------------------------------------------
# Objective and entropy
# ---------------------------------------------------------------------------

def objective(gx: Grid, gy: Grid, T, eps: float):
    """E(T) = sum_{ijpq} (dX_ij - dY_pq)^2 T_ip T_jq (Sec. 2) expanded with
    T's own marginals r = T 1, c = T^T 1:
    E = r^T (D_X o D_X) r + c^T (D_Y o D_Y) c - 2 <D_X T D_Y, T>.
    Returns (E, E + eps * H(T)), H = sum T (ln T - 1), 0 ln 0 = 0."""
    T = np.asarray(T, dtype=np.float64)
    DX, DY = cost_matrix(gx), cost_matrix(gy)
    r = T.sum(axis=1)
    c = T.sum(axis=0)
    E = r @ ((DX * DX) @ r) + c @ ((DY * DY) @ c) - 2.0 * np.sum(((DX @ T) @ DY) * T)
    return float(E), float(E + eps * entropy(T))


def entropy(T) -> float:
    T = np.asarray(T, dtype=np.float64)
    pos = T > 0
    return float(np.sum(T[pos] * (np.log(T[pos]) - 1.0)))


# ---------------------------------------------------------------------------
# Log-domain Sinkhorn (the entropic OT sub-problem of the mirror-descent step)
# ---------------------------------------------------------------------------

def _lse_last_axis(Z: np.ndarray) -> np.ndarray:
    """log sum exp along the last axis, shifted by the maximum; -inf entries
    contribute nothing; an all -inf line gives -inf."""
    m = np.max(Z, axis=-1)
    safe = np.where(np.isfinite(m), m, 0.0)
    s = np.sum(np.exp(Z - safe[..., None]), axis=-1)
    with np.errstate(divide="ignore"):
        out = safe + np.log(s)
    return np.where(np.isneginf(m), -np.inf, out)


def sinkhorn(C, p, q, eps: float, iters: int, f0=None, g0=None):
    """Entropic OT  min <C, P> + eps H(P)  over the couplings of (p, q).

    Potentials start at zero (or at f0, g0 when warm-started).  One iteration
    is f_i = eps ln p_i - eps LSE_p((g_p - C_ip)/eps), then
    g_p = eps ln q_p - eps LSE_i((f_i - C_ip)/eps) with the new f.
    Zero-mass entries get -inf directly.  Returns (f, g)."""
    C = np.asarray(C, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    M, N = C.shape
    f = np.zeros(M) if f0 is None else np.array(f0, dtype=np.float64)
    g = np.zeros(N) if g0 is None else np.array(g0, dtype=np.float64)
    with np.errstate(divide="ignore"):
        logp, logq = np.log(p), np.log(q)
    for _ in range(iters):
        f = eps * logp - eps * _lse_last_axis((g[None, :] - C) / eps)
        f[p == 0] = -np.inf
        g = eps * logq - eps * _lse_last_axis(((f[:, None] - C) / eps).T)
        g[q == 0] = -np.inf
    return f, g


def sinkhorn_tol(C, p, q, eps: float, max_iters: int, check_every: int, tol: float,
                 f0=None, g0=None):
    """Sinkhorn with a stopping rule (the paper runs fixed iteration counts and
    states none; this is the reading taken for tolerance-based stopping).

    Iteration t (1-based) is the update of ``sinkhorn``.  When t is a multiple
    of check_every, the plan (f_t, g_{t-1}) of the half-step -- its row sums are
    p after the f update -- has its column-marginal violation
    err_t = sum_p |sum_i P_ip - q_p| measured; the g update of iteration t is
    still applied, and if err_t <= tol the iteration stops there.
    Returns (f, g, iterations done, last measured err or nan)."""
    C = np.asarray(C, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    M, N = C.shape
    f = np.zeros(M) if f0 is None else np.array(f0, dtype=np.float64)
    g = np.zeros(N) if g0 is None else np.array(g0, dtype=np.float64)
    with np.errstate(divide="ignore"):
        logp, logq = np.log(p), np.log(q)
    err = float("nan")
    for t in range(1, max_iters + 1):
        f = eps * logp - eps * _lse_last_axis((g[None, :] - C) / eps)
        f[p == 0] = -np.inf
        check = t % check_every == 0
        if check:
            col = plan(C, f, g, eps).sum(axis=0)
            err = float(np.sum(np.abs(col - q)))
        g = eps * logq - eps * _lse_last_axis(((f[:, None] - C) / eps).T)
        g[q == 0] = -np.inf
        if check and err <= tol:
            return f, g, t, err
    return f, g, max_iters, err


def plan(C, f, g, eps: float) -> np.ndarray:
    """P_ip = exp((f_i + g_p - C_ip)/eps)."""
    C = np.asarray(C, dtype=np.float64)
    return np.exp((np.asarray(f)[:, None] + np.asarray(g)[None, :] - C) / eps)


# ---------------------------------------------------------------------------
# Mirror descent (entropic GW), tau = eps
# ---------------------------------------------------------------------------

def solve(gx: Grid, gy: Grid, p, q, eps: float, outer: int, inner: int,
          gradient: str = "dense", warm: bool = False):
    """T^0 = p q^T; each outer step computes G(T^l), runs Sinkhorn on the cost
    2G (= the paper's gradient, Remark tau = eps) and sets T^{l+1} to its plan.
    Returns (T, f, g, (E, E + eps H))."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    grad = grad_dense if gradient == "dense" else grad_pascal
    T = p[:, None] * q[None, :]
    f = g = None
    for _ in range(outer):
        C = 2.0 * grad(gx, gy, p, q, T)
        if warm and f is not None:
            f, g = sinkhorn(C, p, q, eps, inner, f, g)
        else:
            f, g = sinkhorn(C, p, q, eps, inner)
        T = plan(C, f, g, eps)
    if f is None:
        f, g = np.zeros(p.shape[0]), np.zeros(q.shape[0])
    return T, f, g, objective(gx, gy, T, eps)


def solve_tol(gx: Grid, gy: Grid, p, q, eps: float, outer: int, max_inner: int,
              check_every: int, tol: float, warm: bool = False):
    """``solve`` with each Sinkhorn call stopped by ``sinkhorn_tol``.
    Returns (T, f, g, (E, E + eps H), inner iterations done per outer step)."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    T = p[:, None] * q[None, :]
    f = g = None
    done = []
    for _ in range(outer):
        C = 2.0 * grad_dense(gx, gy, p, q, T)
        if warm and f is not None:
            f, g, k, _ = sinkhorn_tol(C, p, q, eps, max_inner, check_every, tol, f, g)
        else:
            f, g, k, _ = sinkhorn_tol(C, p, q, eps, max_inner, check_every, tol)
        done.append(k)
        T = plan(C, f, g, eps)
    if f is None:
        f, g = np.zeros(p.shape[0]), np.zeros(q.shape[0])
    return T, f, g, objective(gx, gy, T, eps), done


# ---------------------------------------------------------------------------
# Fused GW (Remark, Entropic algorithm for FGW)
# ---------------------------------------------------------------------------

def feature_cost_sq(fa, fb) -> np.ndarray:
    """c_ip^2 with c_ip = fa_i - fb_p."""
    fa = np.asarray(fa, dtype=np.float64)
    fb = np.asarray(fb, dtype=np.float64)
    d = fa[:, None] - fb[None, :]
    return d * d


def grad_fgw(gx: Grid, gy: Grid, p, q, T, fa, fb, theta: float) -> np.ndarray:
    """Half of the FGW gradient: the Remark gives
    grad = (1 - theta) C o C + theta * grad E (C_2 - 4 theta D T D with
    C_2 = (1 - theta) C o C + 2 theta (constant terms)), and G = grad E / 2, so
    the value here is theta G + (1 - theta) / 2 C o C."""
    G = grad_dense(gx, gy, p, q, T)
    return theta * G + 0.5 * (1.0 - theta) * feature_cost_sq(fa, fb)


def objective_fgw(gx: Grid, gy: Grid, T, fa, fb, theta: float, eps: float):
    """(1 - theta) sum c_ip^2 T_ip + theta E(T) (the Remark's objective), and
    the same plus eps H(T)."""
    T = np.asarray(T, dtype=np.float64)
    E, _ = objective(gx, gy, T, eps)
    Ef = (1.0 - theta) * float(np.sum(feature_cost_sq(fa, fb) * T)) + theta * E
    return float(Ef), float(Ef + eps * entropy(T))


def solve_fgw(gx: Grid, gy: Grid, p, q, fa, fb, theta: float, eps: float, outer: int,
              inner: int, warm: bool = False):
    """Mirror descent of the Remark: the iteration of Eq. (GW sinkhorn) with the
    FGW gradient as the cost (tau = eps).  T^0 = p q^T.
    Returns (T, f, g, (E_fgw, E_fgw + eps H))."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    T = p[:, None] * q[None, :]
    f = g = None
    for _ in range(outer):
        C = 2.0 * grad_fgw(gx, gy, p, q, T, fa, fb, theta)
        if warm and f is not None:
            f, g = sinkhorn(C, p, q, eps, inner, f, g)
        else:
            f, g = sinkhorn(C, p, q, eps, inner)
        T = plan(C, f, g, eps)
    if f is None:
        f, g = np.zeros(p.shape[0]), np.zeros(q.shape[0])
    return T, f, g, objective_fgw(gx, gy, T, fa, fb, theta, eps)


# ---------------------------------------------------------------------------
# Unbalanced GW (Remark, Entropic algorithm for UGW)
# ---------------------------------------------------------------------------
# The Remark fixes the divergence and the sub-problem solved at each step,
#   min_{T >= 0} < G(Th) + g(Th), T > + m(Th) (rho KL(T 1 | u) + rho KL(T^T 1 | v)
#                                            + eps KL(T | u (x) v)),
# with G(Th) = grad E(Th) / 2 taken with Th's own marginals, but not the scalar
# g(Th) nor the solver of the sub-problem; both are read from the UGW work the
# Remark cites (alternate minimisation of its bi-convex relaxation):
#   g(Th) = rho <log(a/u), a> + rho <log(b/v), b> + eps <log(Th/(u (x) v)), Th>,
#           a = Th 1, b = Th^T 1;
#   the sub-problem by unbalanced Sinkhorn on the dual potentials,
#           f = -tau e LSE_p((g_p - C_ip)/e + ln v_p),
#           g = -tau e LSE_i((f_i - C_ip)/e + ln u_i),
#           tau = r / (r + e),  r = m(Th) rho,  e = m(Th) eps,
#           T_ip = exp((f_i + g_p - C_ip)/e) u_i v_p;
#   then the mass is rescaled, T <- sqrt(m(Th) / m(T)) T, and
#   T^0 = u (x) v / sqrt(m(u) m(v)).
# KL is the divergence of positive measures, KL(a|b) = sum a log(a/b) - m(a) + m(b),
# and the quadratic one KL(a (x) a | b (x) b) = 2 m(a) KL(a|b) + (m(a) - m(b))^2.

def mass(a) -> float:
    return float(np.sum(np.asarray(a, dtype=np.float64)))


def kl(a, b) -> float:
    """KL(a|b) = sum a log(a/b) - m(a) + m(b) for non-negative a, b (0 log 0 = 0)."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    pos = a > 0
    return float(np.sum(a[pos] * np.log(a[pos] / b[pos])) - a.sum() + b.sum())


def quad_kl(a, b) -> float:
    """KL(a (x) a | b (x) b), by the identity 2 m(a) KL(a|b) + (m(a) - m(b))^2."""
    return 2.0 * mass(a) * kl(a, b) + (mass(a) - mass(b)) ** 2


def ugw_shift(T, u, v, rho: float, eps: float) -> float:
    """g(T) = rho <log(a/u), a> + rho <log(b/v), b> + eps <log(T/(u (x) v)), T>."""
    T = np.asarray(T, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    a, b = T.sum(axis=1), T.sum(axis=0)

    def xlogy(x, y):
        pos = x > 0
        return float(np.sum(x[pos] * np.log(x[pos] / y[pos])))

    return (rho * xlogy(a, u) + rho * xlogy(b, v)
            + eps * xlogy(T, u[:, None] * v[None, :]))


def uot_sinkhorn(C, u, v, rho: float, eps: float, iters: int, f0=None, g0=None):
    """Unbalanced entropic OT, min <C, T> + rho KL(T1|u) + rho KL(T^T 1|v)
    + eps KL(T|u (x) v), by the log-domain potential updates (f then g).
    Returns (f, g)."""
    C = np.asarray(C, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    M, N = C.shape
    tau = rho / (rho + eps)
    with np.errstate(divide="ignore"):
        lu, lv = np.log(u), np.log(v)
    f = np.zeros(M) if f0 is None else np.array(f0, dtype=np.float64)
    g = np.zeros(N) if g0 is None else np.array(g0, dtype=np.float64)
    for _ in range(iters):
        f = -tau * eps * _lse_last_axis((g[None, :] - C) / eps + lv[None, :])
        g = -tau * eps * _lse_last_axis(((f[:, None] - C) / eps + lu[:, None]).T)
    return f, g


def uot_plan(C, f, g, u, v, eps: float) -> np.ndarray:
    """T_ip = exp((f_i + g_p - C_ip)/eps) u_i v_p."""
    C = np.asarray(C, dtype=np.float64)
    return (np.exp((np.asarray(f)[:, None] + np.asarray(g)[None, :] - C) / eps)
            * np.asarray(u, dtype=np.float64)[:, None] * np.asarray(v, dtype=np.float64)[None, :])


def objective_ugw(gx: Grid, gy: Grid, T, u, v, rho: float, eps: float):
    """The Remark's divergence E(T) + rho KL(a (x) a|u (x) u) + rho KL(b (x) b|v (x) v)
    (E with T's own marginals), and the same plus eps KL(T (x) T|(u (x) v) (x) (u (x) v))."""
    T = np.asarray(T, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    E, _ = objective(gx, gy, T, 0.0)
    U = E + rho * quad_kl(T.sum(axis=1), u) + rho * quad_kl(T.sum(axis=0), v)
    return float(U), float(U + eps * quad_kl(T, u[:, None] * v[None, :]))


def solve_ugw(gx: Grid, gy: Grid, u, v, rho: float, eps: float, outer: int, inner: int):
    """Entropic UGW by the Remark's iteration (readings above).
    Returns (T, f, g, objective_ugw(T))."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    T = u[:, None] * v[None, :] / math.sqrt(mass(u) * mass(v))
    f, g = np.zeros(u.shape[0]), np.zeros(v.shape[0])
    for _ in range(outer):
        m = mass(T)
        a, b = T.sum(axis=1), T.sum(axis=0)
        C = grad_dense(gx, gy, a, b, T) + ugw_shift(T, u, v, rho, eps)
        e = m * eps
        f, g = uot_sinkhorn(C, u, v, m * rho, e, inner)
        P = uot_plan(C, f, g, u, v, e)
        T = math.sqrt(m / mass(P)) * P
    return T, f, g, objective_ugw(gx, gy, T, u, v, rho, eps)
