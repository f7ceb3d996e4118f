"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, sizes workspaces and rejects invalid arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gw.h")
LIB = os.path.join(ROOT, "paper_2404_08970_amd", "libgw.so")



@pytest.fixture(scope="module", autouse=True)
def _built_library():
    """The checks need the library itself: build it when it is not there yet
    (hipcc cross-compiles for gfx950 without a GPU)."""
    if not os.path.exists(LIB):
        from paper_2404_08970_amd import build_lib
        build_lib.build()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**(gw_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_three_calls():
    names = declared_functions()
    for n in ("gw_grad", "gw_sinkhorn", "gw_solve"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def _gw():
    from paper_2404_08970_amd import gw
    return gw


def test_status_strings():
    gw = _gw()
    lib = gw.library()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.gw_status_string(code).decode().startswith("GW_")
    assert b"gfx950" in lib.gw_version()


def test_workspace_bytes_arithmetic():
    gw = _gw()
    X = gw.Grid((4096,), 1 / 4095, 2)
    Y = gw.Grid((4096,), 1 / 4095, 2)
    fast = gw.workspace_bytes(X, Y, gw.PATH_FAST_F64, gw.OP_GRAD)
    dense = gw.workspace_bytes(X, Y, gw.PATH_DENSE_F64, gw.OP_GRAD)
    solve = gw.workspace_bytes(X, Y, gw.PATH_FAST_F64, gw.OP_SOLVE)
    MN8 = 4096 * 4096 * 8
    # FAST keeps only O(MN k / 64) of carries: row moments, column moments and the
    # D~_Y-applied column carries, each 2 (k + 1) values per line per 64-wide tile,
    # plus c1 and c2; dense needs the full intermediate product
    carries = 3 * 2 * (2 + 1) * (4096 // 64) * 4096 * 8
    assert carries <= fast <= carries + 2 * 4096 * 8 + 4 * 256
    assert fast < MN8 // 2
    assert dense >= MN8
    assert solve >= MN8            # the gradient buffer of the solve
    assert fast % 256 == 0 and solve % 256 == 0
    bad = gw.Grid((4096,), 1 / 4095, 9)
    assert gw.workspace_bytes(bad, Y, gw.PATH_FAST_F64, gw.OP_GRAD) == 0


def _call_grad(gw, X, Y, p=8, q=8, T=8, ldT=None, G=64, ldG=None, path=0, ws=256, nbytes=1 << 30):
    xc, yc = X.c(), Y.c()
    N = Y.size
    return gw.library().gw_grad(ctypes.byref(xc), ctypes.byref(yc), ctypes.c_void_p(p),
                                ctypes.c_void_p(q), ctypes.c_void_p(T), ldT or N,
                                ctypes.c_void_p(G), ldG or N, path, ctypes.c_void_p(ws), nbytes,
                                ctypes.c_void_p(0))


def test_invalid_arguments_rejected_before_launch():
    gw = _gw()
    X = gw.Grid((16,), 1.0, 1)
    Y = gw.Grid((16,), 1.0, 1)
    big = 1 << 40  # fake, never dereferenced: validation fails first
    EINVAL, ENOMEM = gw.GW_EINVAL, gw.GW_ENOMEM
    assert _call_grad(gw, X, Y, p=0, T=big, G=2 * big) == EINVAL              # null p
    assert _call_grad(gw, X, Y, p=big + 4, T=big, G=2 * big) == EINVAL        # misaligned
    assert _call_grad(gw, X, Y, p=big, q=big, T=big, G=2 * big, ldT=8) == EINVAL  # ld < N
    assert _call_grad(gw, X, Y, p=big, q=big, T=big, G=big + 8) == EINVAL     # G overlaps T
    assert _call_grad(gw, X, Y, p=big, q=big, T=big, G=2 * big, path=9) == EINVAL
    assert _call_grad(gw, X, Y, p=big, q=big, T=big, G=2 * big, nbytes=16) == ENOMEM
    assert _call_grad(gw, X, Y, p=big, q=big, T=big, G=2 * big, ws=big + 8) == EINVAL
    for bad in (gw.Grid((16,), 0.0, 1), gw.Grid((16,), 1.0, 0), gw.Grid((16,), 1.0, 5),
                gw.Grid((0,), 1.0, 1), gw.Grid((4, 4), 1.0, 3, gw.METRIC_SQEUCLID),
                gw.Grid((16,), float("nan"), 1)):
        assert _call_grad(gw, bad, Y, p=big, q=big, T=big, G=2 * big) == EINVAL


def test_sinkhorn_and_solve_validation():
    gw = _gw()
    lib = gw.library()
    big = 1 << 40
    P = ctypes.c_void_p
    # eps <= 0
    st = lib.gw_sinkhorn(P(big), 16, 16, 16, 1.0, P(big), P(big), 0.0, 10, 1, P(big), P(big),
                         P(0), 16, P(big), 1 << 30, P(0))
    assert st == gw.GW_EINVAL
    # rows longer than the largest extent (65535)
    st = lib.gw_sinkhorn(P(big), 70000, 4, 70000, 1.0, P(big), P(big), 0.1, 10, 1, P(big),
                         P(big), P(0), 70000, P(big), 1 << 40, P(0))
    assert st == gw.GW_EUNSUPPORTED
    X = gw.Grid((16,), 1.0, 1)
    xc = X.c()
    st = lib.gw_solve(ctypes.byref(xc), ctypes.byref(xc), P(big), P(big), 0.1, -1, 10, 0, 0,
                      P(big), 16, P(big), P(big), P(0), P(big), 1 << 30, P(0))
    assert st == gw.GW_EINVAL
    st = lib.gw_solve(ctypes.byref(xc), ctypes.byref(xc), P(big), P(big), 0.1, 1, 10, 0, 8,
                      P(big), 16, P(big), P(big), P(0), P(big), 1 << 30, P(0))
    assert st == gw.GW_EINVAL        # unknown flag
