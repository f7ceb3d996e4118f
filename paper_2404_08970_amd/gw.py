"""Python binding of libgw.so (argument marshalling only).

Every computation runs in the HIP kernels of ``libgw.so``; this module checks
tensor placement, allocates the caller-owned workspace with PyTorch and passes
raw device pointers plus the current HIP stream.  If the library has not been
built, importing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import time
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgw.so")

GW_OK, GW_EINVAL, GW_ENOMEM, GW_EDEVICE, GW_ENUMERIC, GW_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
GW_EAGAIN = -6
METRIC_L1POW, METRIC_SQEUCLID = 0, 1
PATH_FAST_F64, PATH_DENSE_F64, PATH_DENSE_F32, PATH_DENSE_BF16 = 0, 1, 2, 3
PATH_DENSE_BF16_SPLIT, PATH_DENSE_F32_SPLIT = 4, 5
OP_GRAD, OP_SINKHORN, OP_SOLVE, OP_OBJECTIVE, OP_UOT_SINKHORN, OP_SOLVE_UGW = 0, 1, 2, 3, 4, 5
FLAG_WARM_START = 1
REQ_OBJECTIVE = 2
REQ_QUEUED, REQ_RUNNING, REQ_DONE = 0, 1, 2
KMAX = 4

PATHS = {
    "fast": PATH_FAST_F64, "fast_f64": PATH_FAST_F64,
    "dense": PATH_DENSE_F64, "dense_f64": PATH_DENSE_F64,
    "dense_f32": PATH_DENSE_F32, "dense_bf16": PATH_DENSE_BF16,
    "dense_bf16_split": PATH_DENSE_BF16_SPLIT, "dense_f32_split": PATH_DENSE_F32_SPLIT,
}

# timing families (gw.h)
(FAM_FAST_MAIN, FAM_FAST_CARRY, FAM_DENSE, FAM_SINK_ROW, FAM_SINK_COL, FAM_PLAN, FAM_OTHER, FAM_2D,
 FAM_SERVE_STEP) = range(9)


class GWError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {_lib().gw_status_string(status).decode()} ({status})")
        self.status = status


class c_grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("k", ctypes.c_int32), ("metric", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("shape", ctypes.c_int64 * 3), ("h", ctypes.c_double)]


class c_request(ctypes.Structure):
    _fields_ = [("X", c_grid), ("Y", c_grid), ("p", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("eps", ctypes.c_double), ("outer", ctypes.c_int32), ("inner", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class c_result(ctypes.Structure):
    _fields_ = [("T", ctypes.c_void_p), ("f", ctypes.c_void_p), ("g", ctypes.c_void_p),
                ("M", ctypes.c_int64), ("N", ctypes.c_int64), ("obj", ctypes.c_double * 2),
                ("done_ms", ctypes.c_double), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_LIB = None


def _lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2404_08970_amd.build_lib` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    G = ctypes.POINTER(c_grid)
    lib.gw_workspace_bytes.argtypes = [G, G, I32, I32]
    lib.gw_workspace_bytes.restype = SZ
    lib.gw_grad.argtypes = [G, G, P, P, P, I64, P, I64, I32, P, SZ, P]
    lib.gw_grad.restype = I32
    lib.gw_sinkhorn.argtypes = [P, I64, I64, I64, D, P, P, D, I32, I32, P, P, P, I64, P, SZ, P]
    lib.gw_sinkhorn.restype = I32
    lib.gw_sinkhorn_noalloc.argtypes = [P, I64, I64, I64, D, P, P, D, I32, I32, P, P, P, I64, P]
    lib.gw_sinkhorn_noalloc.restype = I32
    lib.gw_solve.argtypes = [G, G, P, P, D, I32, I32, I32, I32, P, I64, P, P, P, P, SZ, P]
    lib.gw_solve.restype = I32
    lib.gw_objective.argtypes = [G, G, P, I64, D, P, P, SZ, P]
    lib.gw_objective.restype = I32
    lib.gw_sinkhorn_tol.argtypes = [P, I64, I64, I64, D, P, P, D, I32, I32, D, I32, P, P, P, I64,
                                    P, P, P, SZ, P]
    lib.gw_sinkhorn_tol.restype = I32
    lib.gw_solve_tol.argtypes = [G, G, P, P, D, I32, I32, I32, D, I32, I32, P, I64, P, P, P, P, P,
                                 SZ, P]
    lib.gw_solve_tol.restype = I32
    lib.gw_uot_sinkhorn.argtypes = [P, I64, I64, I64, D, P, P, D, D, I32, I32, P, P, P, I64, P,
                                    SZ, P]
    lib.gw_uot_sinkhorn.restype = I32
    lib.gw_solve_ugw.argtypes = [G, G, P, P, D, D, I32, I32, I32, P, I64, P, P, P, P, SZ, P]
    lib.gw_solve_ugw.restype = I32
    lib.gw_grad_fgw.argtypes = [G, G, P, P, P, P, D, P, I64, P, I64, I32, P, SZ, P]
    lib.gw_grad_fgw.restype = I32
    lib.gw_solve_fgw.argtypes = [G, G, P, P, P, P, D, D, I32, I32, I32, I32, P, I64, P, P, P, P,
                                 SZ, P]
    lib.gw_solve_fgw.restype = I32
    lib.gw_objective_fgw.argtypes = [G, G, P, I64, P, P, D, D, P, P, SZ, P]
    lib.gw_objective_fgw.restype = I32
    lib.gw_status_string.argtypes = [I32]
    lib.gw_status_string.restype = ctypes.c_char_p
    lib.gw_check_status.argtypes = [P, P]
    lib.gw_check_status.restype = I32
    lib.gw_profile_enable.argtypes = [I32]
    lib.gw_profile_enable.restype = None
    lib.gw_profile_read.argtypes = [I32, ctypes.POINTER(D), ctypes.POINTER(I64)]
    lib.gw_profile_read.restype = I32
    lib.gw_profile_sample.argtypes = [I32]
    lib.gw_profile_sample.restype = I32
    lib.gw_version.argtypes = []
    lib.gw_version.restype = ctypes.c_char_p
    R, PS = ctypes.POINTER(c_request), ctypes.POINTER(ctypes.c_void_p)
    lib.gw_server_request_bytes.argtypes = [R]
    lib.gw_server_request_bytes.restype = SZ
    lib.gw_server_table_bytes.argtypes = [I32]
    lib.gw_server_table_bytes.restype = SZ
    lib.gw_server_create.argtypes = [P, SZ, I32, I32, P, PS]
    lib.gw_server_create.restype = I32
    lib.gw_server_set_boost.argtypes = [P, I32]
    lib.gw_server_set_boost.restype = I32
    lib.gw_server_submit.argtypes = [P, R, ctypes.POINTER(I64)]
    lib.gw_server_submit.restype = I32
    lib.gw_server_step.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.gw_server_step.restype = I32
    lib.gw_server_poll.argtypes = [P, I64, ctypes.POINTER(I32)]
    lib.gw_server_poll.restype = I32
    lib.gw_server_result.argtypes = [P, I64, ctypes.POINTER(c_result)]
    lib.gw_server_result.restype = I32
    lib.gw_server_release.argtypes = [P, I64]
    lib.gw_server_release.restype = I32
    lib.gw_server_destroy.argtypes = [P]
    lib.gw_server_destroy.restype = I32
    _LIB = lib
    return lib


def library():
    """The loaded ctypes library (raises if it is not built)."""
    return _lib()


@dataclass(frozen=True)
class Grid:
    """Uniform grid: ``shape=(n,)`` (1D), ``(H, W)`` (2D) or ``(D, H, W)`` (3D),
    flattened row-major."""
    shape: tuple
    h: float
    k: int
    metric: int = METRIC_L1POW

    @property
    def ndim(self):
        return len(self.shape)

    @property
    def size(self):
        n = 1
        for s in self.shape:
            n *= int(s)
        return n

    def c(self) -> c_grid:
        g = c_grid()
        g.ndim = self.ndim
        g.k = self.k
        g.metric = self.metric
        g.reserved = 0
        g.shape[0] = int(self.shape[0])
        g.shape[1] = int(self.shape[1]) if self.ndim >= 2 else 1
        g.shape[2] = int(self.shape[2]) if self.ndim == 3 else 1
        g.h = float(self.h)
        return g


def unit_grid(shape, k: int, metric: int = METRIC_L1POW) -> Grid:
    """Grid on [0,1] along its first axis (the other axes share the spacing),
    h = 1/(n-1)."""
    shape = tuple(int(s) for s in shape)
    h = 1.0 / max(shape[0] - 1, 1)
    return Grid(shape, h, k, metric)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_f64(name, t, shape=None):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
        raise TypeError(f"{name} must be a CUDA float64 tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.dim() == 2:
        if t.stride(1) != 1:
            raise ValueError(f"{name} must be row-major with unit column stride")
    elif t.dim() == 1 and t.stride(0) != 1:
        raise ValueError(f"{name} must be contiguous")


_WS_CACHE = {}


def workspace(nbytes: int, device=None, key="default") -> torch.Tensor:
    """A 256-byte aligned device workspace of at least ``nbytes`` (cached)."""
    dev = torch.device("cuda") if device is None else torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    ck = (key, idx)
    buf = _WS_CACHE.get(ck)
    if buf is None or buf.numel() < nbytes + 256:
        buf = torch.empty(max(nbytes, 1) + 256, dtype=torch.uint8, device=f"cuda:{idx}")
        _WS_CACHE[ck] = buf
    off = (-buf.data_ptr()) % 256
    return buf[off:off + max(nbytes, 1)]


def workspace_bytes(X: Grid, Y: Grid, path=PATH_FAST_F64, op=OP_GRAD) -> int:
    xc, yc = X.c(), Y.c()
    return int(_lib().gw_workspace_bytes(ctypes.byref(xc), ctypes.byref(yc), int(path), int(op)))


def _raise(st, what):
    if st != GW_OK:
        raise GWError(st, what)


def grad(X: Grid, Y: Grid, p, q, T, path=PATH_FAST_F64, out=None, ws=None):
    """G = c1 1^T + 1 c2^T - 2 D_X T D_Y on the GPU."""
    path = PATHS.get(path, path)
    M, N = X.size, Y.size
    _check_f64("p", p, (M,)); _check_f64("q", q, (N,)); _check_f64("T", T, (M, N))
    if out is None:
        out = torch.empty((M, N), dtype=torch.float64, device=T.device)
    _check_f64("out", out, (M, N))
    nb = workspace_bytes(X, Y, path, OP_GRAD)
    if nb == 0:
        raise GWError(GW_EINVAL, "gw_workspace_bytes")
    if ws is None:
        ws = workspace(nb, T.device)
    xc, yc = X.c(), Y.c()
    st = _lib().gw_grad(ctypes.byref(xc), ctypes.byref(yc), _ptr(p), _ptr(q), _ptr(T), T.stride(0),
                        _ptr(out), out.stride(0), int(path), _ptr(ws), ws.numel(), _stream())
    _raise(st, "gw_grad")
    return out


def sinkhorn(C, p, q, eps: float, iters: int, c_scale: float = 1.0, f=None, g=None,
             plan: bool = False, ws=None):
    """Log-domain Sinkhorn on the GPU; returns (f, g) or (f, g, T)."""
    M, N = C.shape
    _check_f64("C", C, (M, N)); _check_f64("p", p, (M,)); _check_f64("q", q, (N,))
    init_zero = 1 if (f is None and g is None) else 0
    if f is None:
        f = torch.zeros(M, dtype=torch.float64, device=C.device)
    if g is None:
        g = torch.zeros(N, dtype=torch.float64, device=C.device)
    T = torch.empty((M, N), dtype=torch.float64, device=C.device) if plan else None
    gx, gy = Grid((M,), 1.0, 1), Grid((N,), 1.0, 1)
    nb = workspace_bytes(gx, gy, PATH_FAST_F64, OP_SINKHORN)
    if ws is None:
        ws = workspace(nb, C.device)
    st = _lib().gw_sinkhorn(_ptr(C), C.stride(0), M, N, float(c_scale), _ptr(p), _ptr(q),
                            float(eps), int(iters), init_zero, _ptr(f), _ptr(g), _ptr(T),
                            T.stride(0) if T is not None else N, _ptr(ws), ws.numel(), _stream())
    _raise(st, "gw_sinkhorn")
    return (f, g, T) if plan else (f, g)


def sinkhorn_noalloc(C, p, q, eps: float, iters: int, c_scale: float = 1.0, f=None, g=None,
                     T=None):
    """gw_sinkhorn_noalloc: the Sinkhorn call whose scratch is the library's
    static device array (no workspace).  f, g (and T for the plan) are caller
    buffers; missing f, g are allocated here by torch before the call, which
    itself allocates nothing.  Returns (f, g) or (f, g, T)."""
    M, N = C.shape
    _check_f64("C", C, (M, N)); _check_f64("p", p, (M,)); _check_f64("q", q, (N,))
    init_zero = 1 if (f is None and g is None) else 0
    if f is None:
        f = torch.zeros(M, dtype=torch.float64, device=C.device)
    if g is None:
        g = torch.zeros(N, dtype=torch.float64, device=C.device)
    if T is not None:
        _check_f64("T", T, (M, N))
    st = _lib().gw_sinkhorn_noalloc(_ptr(C), C.stride(0), M, N, float(c_scale), _ptr(p), _ptr(q),
                                    float(eps), int(iters), init_zero, _ptr(f), _ptr(g), _ptr(T),
                                    T.stride(0) if T is not None else N, _stream())
    _raise(st, "gw_sinkhorn_noalloc")
    return (f, g, T) if T is not None else (f, g)


def sinkhorn_tol(C, p, q, eps: float, max_iters: int, check_every: int, tol: float,
                 c_scale: float = 1.0, f=None, g=None, plan: bool = False, ws=None):
    """Sinkhorn stopped once the column violation of the half-step plan, measured
    every check_every iterations, is <= tol.  Returns (f, g, iters_done, err) or
    (f, g, T, iters_done, err); iters_done (int32) and err are device tensors."""
    M, N = C.shape
    _check_f64("C", C, (M, N)); _check_f64("p", p, (M,)); _check_f64("q", q, (N,))
    init_zero = 1 if (f is None and g is None) else 0
    if f is None:
        f = torch.zeros(M, dtype=torch.float64, device=C.device)
    if g is None:
        g = torch.zeros(N, dtype=torch.float64, device=C.device)
    T = torch.empty((M, N), dtype=torch.float64, device=C.device) if plan else None
    done = torch.empty(1, dtype=torch.int32, device=C.device)
    err = torch.empty(1, dtype=torch.float64, device=C.device)
    gx, gy = Grid((M,), 1.0, 1), Grid((N,), 1.0, 1)
    nb = workspace_bytes(gx, gy, PATH_FAST_F64, OP_SINKHORN)
    if ws is None:
        ws = workspace(nb, C.device)
    st = _lib().gw_sinkhorn_tol(_ptr(C), C.stride(0), M, N, float(c_scale), _ptr(p), _ptr(q),
                                float(eps), int(max_iters), int(check_every), float(tol),
                                init_zero, _ptr(f), _ptr(g), _ptr(T),
                                T.stride(0) if T is not None else N, _ptr(done), _ptr(err),
                                _ptr(ws), ws.numel(), _stream())
    _raise(st, "gw_sinkhorn_tol")
    return (f, g, T, done, err) if plan else (f, g, done, err)


def solve_tol(X: Grid, Y: Grid, p, q, eps: float, outer: int, max_inner: int, check_every: int,
              tol: float, path=PATH_FAST_F64, warm: bool = False, objective: bool = True,
              T=None, f=None, g=None, obj=None, ws=None):
    """Entropic GW mirror descent whose Sinkhorn calls stop by tolerance; returns
    (T, f, g, obj[2] or None, inner_done[outer] int32 device tensor)."""
    path = PATHS.get(path, path)
    M, N = X.size, Y.size
    _check_f64("p", p, (M,)); _check_f64("q", q, (N,))
    dev = p.device
    T = torch.empty((M, N), dtype=torch.float64, device=dev) if T is None else T
    f = torch.empty(M, dtype=torch.float64, device=dev) if f is None else f
    g = torch.empty(N, dtype=torch.float64, device=dev) if g is None else g
    if objective and obj is None:
        obj = torch.empty(2, dtype=torch.float64, device=dev)
    done = torch.empty(max(int(outer), 1), dtype=torch.int32, device=dev)
    nb = workspace_bytes(X, Y, path, OP_SOLVE)
    if nb == 0:
        raise GWError(GW_EINVAL, "gw_workspace_bytes")
    if ws is None:
        ws = workspace(nb, dev, key="solve")
    xc, yc = X.c(), Y.c()
    st = _lib().gw_solve_tol(ctypes.byref(xc), ctypes.byref(yc), _ptr(p), _ptr(q), float(eps),
                             int(outer), int(max_inner), int(check_every), float(tol), int(path),
                             FLAG_WARM_START if warm else 0, _ptr(T), T.stride(0), _ptr(f),
                             _ptr(g), _ptr(obj if objective else None), _ptr(done), _ptr(ws),
                             ws.numel(), _stream())
    _raise(st, "gw_solve_tol")
    return T, f, g, (obj if objective else None), done[:outer]


def solve(X: Grid, Y: Grid, p, q, eps: float, outer: int, inner: int, path=PATH_FAST_F64,
          warm: bool = False, objective: bool = True, T=None, f=None, g=None, obj=None, ws=None):
    """Entropic GW mirror descent on the GPU; returns (T, f, g, obj[2] or None)."""
    path = PATHS.get(path, path)
    M, N = X.size, Y.size
    _check_f64("p", p, (M,)); _check_f64("q", q, (N,))
    dev = p.device
    T = torch.empty((M, N), dtype=torch.float64, device=dev) if T is None else T
    f = torch.empty(M, dtype=torch.float64, device=dev) if f is None else f
    g = torch.empty(N, dtype=torch.float64, device=dev) if g is None else g
    if objective and obj is None:
        obj = torch.empty(2, dtype=torch.float64, device=dev)
    nb = workspace_bytes(X, Y, path, OP_SOLVE)
    if nb == 0:
        raise GWError(GW_EINVAL, "gw_workspace_bytes")
    if ws is None:
        ws = workspace(nb, dev, key="solve")
    xc, yc = X.c(), Y.c()
    st = _lib().gw_solve(ctypes.byref(xc), ctypes.byref(yc), _ptr(p), _ptr(q), float(eps),
                         int(outer), int(inner), int(path), FLAG_WARM_START if warm else 0,
                         _ptr(T), T.stride(0), _ptr(f), _ptr(g), _ptr(obj if objective else None),
                         _ptr(ws), ws.numel(), _stream())
    _raise(st, "gw_solve")
    return T, f, g, (obj if objective else None)


def objective(X: Grid, Y: Grid, T, eps: float, ws=None):
    """(E(T), E(T) + eps H(T)) as a device tensor of 2 doubles."""
    M, N = X.size, Y.size
    _check_f64("T", T, (M, N))
    obj = torch.empty(2, dtype=torch.float64, device=T.device)
    nb = workspace_bytes(X, Y, PATH_FAST_F64, OP_OBJECTIVE)
    if ws is None:
        ws = workspace(nb, T.device, key="objective")
    xc, yc = X.c(), Y.c()
    st = _lib().gw_objective(ctypes.byref(xc), ctypes.byref(yc), _ptr(T), T.stride(0), float(eps),
                             _ptr(obj), _ptr(ws), ws.numel(), _stream())
    _raise(st, "gw_objective")
    return obj


def uot_sinkhorn(C, u, v, rho: float, eps: float, iters: int, c_shift: float = 0.0, f=None,
                 g=None, plan: bool = False, ws=None):
    """Unbalanced entropic OT on C + c_shift (log-domain potentials); returns
    (f, g) or (f, g, T)."""
    M, N = C.shape
    _check_f64("C", C, (M, N)); _check_f64("u", u, (M,)); _check_f64("v", v, (N,))
    init_zero = 1 if (f is None and g is None) else 0
    if f is None:
        f = torch.zeros(M, dtype=torch.float64, device=C.device)
    if g is None:
        g = torch.zeros(N, dtype=torch.float64, device=C.device)
    T = torch.empty((M, N), dtype=torch.float64, device=C.device) if plan else None
    gx, gy = Grid((M,), 1.0, 1), Grid((N,), 1.0, 1)
    nb = workspace_bytes(gx, gy, PATH_FAST_F64, OP_UOT_SINKHORN)
    if ws is None:
        ws = workspace(nb, C.device, key="uot")
    st = _lib().gw_uot_sinkhorn(_ptr(C), C.stride(0), M, N, float(c_shift), _ptr(u), _ptr(v),
                                float(rho), float(eps), int(iters), init_zero, _ptr(f), _ptr(g),
                                _ptr(T), T.stride(0) if T is not None else N, _ptr(ws),
                                ws.numel(), _stream())
    _raise(st, "gw_uot_sinkhorn")
    return (f, g, T) if plan else (f, g)


def solve_ugw(X: Grid, Y: Grid, u, v, rho: float, eps: float, outer: int, inner: int,
              path=PATH_FAST_F64, objective: bool = True, T=None, f=None, g=None, obj=None,
              ws=None):
    """Entropic unbalanced GW on the GPU; returns (T, f, g, obj[2] or None)."""
    path = PATHS.get(path, path)
    M, N = X.size, Y.size
    _check_f64("u", u, (M,)); _check_f64("v", v, (N,))
    dev = u.device
    T = torch.empty((M, N), dtype=torch.float64, device=dev) if T is None else T
    f = torch.empty(M, dtype=torch.float64, device=dev) if f is None else f
    g = torch.empty(N, dtype=torch.float64, device=dev) if g is None else g
    if objective and obj is None:
        obj = torch.empty(2, dtype=torch.float64, device=dev)
    nb = workspace_bytes(X, Y, path, OP_SOLVE_UGW)
    if nb == 0:
        raise GWError(GW_EINVAL, "gw_workspace_bytes")
    if ws is None:
        ws = workspace(nb, dev, key="ugw")
    xc, yc = X.c(), Y.c()
    st = _lib().gw_solve_ugw(ctypes.byref(xc), ctypes.byref(yc), _ptr(u), _ptr(v), float(rho),
                             float(eps), int(outer), int(inner), int(path), _ptr(T), T.stride(0),
                             _ptr(f), _ptr(g), _ptr(obj if objective else None), _ptr(ws),
                             ws.numel(), _stream())
    _raise(st, "gw_solve_ugw")
    return T, f, g, (obj if objective else None)


def _check_features(fa, fb, M, N):
    _check_f64("fa", fa, (M,)); _check_f64("fb", fb, (N,))


def grad_fgw(X: Grid, Y: Grid, p, q, fa, fb, theta: float, T, path=PATH_FAST_F64, out=None,
             ws=None):
    """Half the fused GW gradient, theta (c1 1^T + 1 c2^T - 2 D_X T D_Y)
    + (1 - theta)/2 (fa_i - fb_p)^2, on the GPU."""
    path = PATHS.get(path, path)
    M, N = X.size, Y.size
    _check_f64("p", p, (M,)); _check_f64("q", q, (N,)); _check_f64("T", T, (M, N))
    _check_features(fa, fb, M, N)
    if out is None:
        out = torch.empty((M, N), dtype=torch.float64, device=T.device)
    _check_f64("out", out, (M, N))
    nb = workspace_bytes(X, Y, path, OP_GRAD)
    if nb == 0:
        raise GWError(GW_EINVAL, "gw_workspace_bytes")
    if ws is None:
        ws = workspace(nb, T.device)
    xc, yc = X.c(), Y.c()
    st = _lib().gw_grad_fgw(ctypes.byref(xc), ctypes.byref(yc), _ptr(p), _ptr(q), _ptr(fa),
                            _ptr(fb), float(theta), _ptr(T), T.stride(0), _ptr(out),
                            out.stride(0), int(path), _ptr(ws), ws.numel(), _stream())
    _raise(st, "gw_grad_fgw")
    return out


def solve_fgw(X: Grid, Y: Grid, p, q, fa, fb, theta: float, eps: float, outer: int, inner: int,
              path=PATH_FAST_F64, warm: bool = False, objective: bool = True, T=None, f=None,
              g=None, obj=None, ws=None):
    """Entropic fused GW mirror descent on the GPU; returns (T, f, g, obj[2] or None)."""
    path = PATHS.get(path, path)
    M, N = X.size, Y.size
    _check_f64("p", p, (M,)); _check_f64("q", q, (N,))
    _check_features(fa, fb, M, N)
    dev = p.device
    T = torch.empty((M, N), dtype=torch.float64, device=dev) if T is None else T
    f = torch.empty(M, dtype=torch.float64, device=dev) if f is None else f
    g = torch.empty(N, dtype=torch.float64, device=dev) if g is None else g
    if objective and obj is None:
        obj = torch.empty(2, dtype=torch.float64, device=dev)
    nb = workspace_bytes(X, Y, path, OP_SOLVE)
    if nb == 0:
        raise GWError(GW_EINVAL, "gw_workspace_bytes")
    if ws is None:
        ws = workspace(nb, dev, key="solve")
    xc, yc = X.c(), Y.c()
    st = _lib().gw_solve_fgw(ctypes.byref(xc), ctypes.byref(yc), _ptr(p), _ptr(q), _ptr(fa),
                             _ptr(fb), float(theta), float(eps), int(outer), int(inner),
                             int(path), FLAG_WARM_START if warm else 0, _ptr(T), T.stride(0),
                             _ptr(f), _ptr(g), _ptr(obj if objective else None), _ptr(ws),
                             ws.numel(), _stream())
    _raise(st, "gw_solve_fgw")
    return T, f, g, (obj if objective else None)


def objective_fgw(X: Grid, Y: Grid, T, fa, fb, theta: float, eps: float, ws=None):
    """(E_fgw(T), E_fgw(T) + eps H(T)) as a device tensor of 2 doubles."""
    M, N = X.size, Y.size
    _check_f64("T", T, (M, N))
    _check_features(fa, fb, M, N)
    obj = torch.empty(2, dtype=torch.float64, device=T.device)
    nb = workspace_bytes(X, Y, PATH_FAST_F64, OP_OBJECTIVE)
    if ws is None:
        ws = workspace(nb, T.device, key="objective")
    xc, yc = X.c(), Y.c()
    st = _lib().gw_objective_fgw(ctypes.byref(xc), ctypes.byref(yc), _ptr(T), T.stride(0),
                                 _ptr(fa), _ptr(fb), float(theta), float(eps), _ptr(obj),
                                 _ptr(ws), ws.numel(), _stream())
    _raise(st, "gw_objective_fgw")
    return obj


def check_status(ws=None):
    """Synchronise and raise if a kernel flagged a non-finite value."""
    st = _lib().gw_check_status(_ptr(ws), _stream())
    _raise(st, "gw_check_status")


def profile_enable(families=None):
    """Record kernel times for the given families (None = all, [] = off)."""
    if families is None:
        mask = 0x1FF
    else:
        mask = 0
        for f in families:
            mask |= 1 << int(f)
    _lib().gw_profile_enable(mask)


def profile_sample(every: int):
    """Time only one launch in `every` of each family (1: all)."""
    _raise(_lib().gw_profile_sample(int(every)), "gw_profile_sample")


def profile_read(family: int):
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _raise(_lib().gw_profile_read(int(family), ctypes.byref(ms), ctypes.byref(n)), "gw_profile_read")
    return ms.value, n.value


# ---------------------------------------------------------------- request loop

def make_request(X: Grid, Y: Grid, p, q, eps: float, outer: int, inner: int,
                 warm: bool = False, objective: bool = False) -> c_request:
    r = c_request()
    r.X, r.Y = X.c(), Y.c()
    r.p, r.q = p.data_ptr() if p is not None else 0, q.data_ptr() if q is not None else 0
    r.eps, r.outer, r.inner = float(eps), int(outer), int(inner)
    r.flags = (FLAG_WARM_START if warm else 0) | (REQ_OBJECTIVE if objective else 0)
    r.reserved = 0
    return r


def request_bytes(X: Grid, Y: Grid, eps: float = 1e-3, outer: int = 1, inner: int = 1) -> int:
    """Arena bytes a request holds while admitted (host arithmetic)."""
    r = make_request(X, Y, None, None, eps, outer, inner)
    r.p = r.q = 256  # any aligned non-null address: only the sizes are read
    return int(_lib().gw_server_request_bytes(ctypes.byref(r)))


class _DeviceView:
    """Exposes a device FP64 buffer through __cuda_array_interface__ (no copy)."""

    def __init__(self, ptr: int, shape):
        self.__cuda_array_interface__ = {"shape": tuple(int(s) for s in shape), "typestr": "<f8",
                                         "data": (int(ptr), False), "version": 2, "strides": None}


class Server:
    """Request loop over a device arena: continuous batching of GW solves.

    ``submit`` queues a solve, ``step`` admits what fits and advances every
    admitted request by one step, ``poll``/``result`` report finished ones and
    ``release`` returns their arena range.  ``p`` and ``q`` tensors are kept
    alive here until release."""

    def __init__(self, arena_bytes: int, max_slots: int = 64, iters_per_step: int = 10,
                 device=None, stream=None, boost: int = 1):
        dev = torch.device("cuda") if device is None else torch.device(device)
        self.device = dev
        self._arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=dev)
        off = (-self._arena.data_ptr()) % 256
        self.arena = self._arena[off:off + int(arena_bytes)]
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p(0)
        st = _lib().gw_server_create(_ptr(self.arena), int(arena_bytes), int(max_slots),
                                     int(iters_per_step), ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(h))
        _raise(st, "gw_server_create")
        self.t0 = time.perf_counter()
        self._h = h
        self._keep = {}
        if boost != 1:
            self.set_boost(boost)

    def set_boost(self, max_boost: int):
        """Size-aware iteration quotas: a request with at most 1/2^m of the
        largest Sinkhorn-phase problem's entries takes 2^m x iters_per_step
        iterations per step (2^m <= max_boost in {1, 2, 4, 8})."""
        _raise(_lib().gw_server_set_boost(self._h, int(max_boost)), "gw_server_set_boost")

    def submit(self, X: Grid, Y: Grid, p, q, eps: float, outer: int, inner: int,
               warm: bool = False, objective: bool = False) -> int:
        _check_f64("p", p, (X.size,)); _check_f64("q", q, (Y.size,))
        r = make_request(X, Y, p, q, eps, outer, inner, warm, objective)
        rid = ctypes.c_int64(0)
        _raise(_lib().gw_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)), "gw_server_submit")
        self._keep[rid.value] = (p, q)
        return rid.value

    def step(self):
        a, qd = ctypes.c_int32(0), ctypes.c_int32(0)
        _raise(_lib().gw_server_step(self._h, ctypes.byref(a), ctypes.byref(qd)), "gw_server_step")
        return a.value, qd.value

    def poll(self, rid: int) -> int:
        s = ctypes.c_int32(0)
        _raise(_lib().gw_server_poll(self._h, int(rid), ctypes.byref(s)), "gw_server_poll")
        return s.value

    def result(self, rid: int, copy: bool = True):
        """dict(T, f, g, obj, done_ms, done_t, status) of a finished request;
        None if it is not finished.  With copy=False T, f, g are views of the
        arena, valid until release."""
        res = c_result()
        st = _lib().gw_server_result(self._h, int(rid), ctypes.byref(res))
        if st == GW_EAGAIN:
            return None
        _raise(st, "gw_server_result")
        M, N = res.M, res.N
        with torch.cuda.device(self.device):
            T = torch.as_tensor(_DeviceView(res.T, (M, N)), device=self.device)
            f = torch.as_tensor(_DeviceView(res.f, (M,)), device=self.device)
            g = torch.as_tensor(_DeviceView(res.g, (N,)), device=self.device)
        if copy:
            with torch.cuda.stream(self.stream):
                T, f, g = T.clone(), f.clone(), g.clone()
        return {"T": T, "f": f, "g": g, "obj": (res.obj[0], res.obj[1]), "done_ms": res.done_ms,
                "done_t": self.t0 + res.done_ms / 1e3, "status": res.status}

    def release(self, rid: int):
        _raise(_lib().gw_server_release(self._h, int(rid)), "gw_server_release")
        self._keep.pop(int(rid), None)

    def close(self):
        if self._h:
            st = _lib().gw_server_destroy(self._h)
            self._h = None
            self._keep.clear()
            _raise(st, "gw_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def server_table_bytes(max_slots: int) -> int:
    return int(_lib().gw_server_table_bytes(int(max_slots)))
