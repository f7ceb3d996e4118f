"""Host-side logic of the request loop (no GPU): the first-fit arena allocator
against a plain Python model, footprint arithmetic and argument validation
that returns before any HIP call."""
import ctypes
import os
import random
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_08970_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "arena_alloc.h"
// stdin: capacity, then lines "a <bytes>" or "r <offset>"; stdout: one line
// per command (offset or FAIL / 1 or 0), then "used largest ranges".
int main() {
  size_t cap;
  if (scanf("%zu", &cap) != 1) return 2;
  gwr::RangeAllocator A(cap);
  char op[4];
  size_t v;
  while (scanf("%3s %zu", op, &v) == 2) {
    if (op[0] == 'a') {
      size_t off = A.alloc(v);
      if (off == gwr::RangeAllocator::kFail) printf("FAIL\n"); else printf("%zu\n", off);
    } else {
      printf("%d\n", A.release(v) ? 1 : 0);
    }
  }
  printf("%zu %zu %zu\n", A.used(), A.largest_free(), A.free_ranges());
  return 0;
}
"""


class ModelAllocator:
    """First fit over a sorted list of free ranges, merged on release."""

    def __init__(self, cap):
        self.free = [(0, cap // 256 * 256)] if cap >= 256 else []
        self.live = {}

    def alloc(self, n):
        n = max(n, 1)
        n = (n + 255) // 256 * 256
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    del self.free[i]
                else:
                    self.free[i] = (off + n, ln - n)
                self.live[off] = n
                return off
        return None

    def release(self, off):
        if off not in self.live:
            return False
        ln = self.live.pop(off)
        self.free.append((off, ln))
        self.free.sort()
        merged = []
        for o, l in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + l)
            else:
                merged.append((o, l))
        self.free = merged
        return True


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("alloc")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_range_allocator_matches_model(driver, seed):
    rng = random.Random(seed)
    cap = 1 << 20
    model = ModelAllocator(cap)
    cmds, expect, live = [], [], []
    for _ in range(600):
        if live and rng.random() < 0.45:
            off = live.pop(rng.randrange(len(live)))
            cmds.append(f"r {off}")
            expect.append("1" if model.release(off) else "0")
        elif rng.random() < 0.03:
            cmds.append("r 12345")  # not a live offset
            expect.append("1" if model.release(12345) else "0")
        else:
            n = rng.choice([1, 255, 256, 257, 4096, rng.randrange(1, 60000)])
            cmds.append(f"a {n}")
            off = model.alloc(n)
            expect.append("FAIL" if off is None else str(off))
            if off is not None:
                live.append(off)
    out = subprocess.run([driver], input=f"{cap}\n" + "\n".join(cmds) + "\n",
                         capture_output=True, text=True, check=True).stdout.split("\n")
    assert out[:len(expect)] == expect
    used = sum(model.live.values())
    largest = max((l for _, l in model.free), default=0)
    assert out[len(expect)] == f"{used} {largest} {len(model.free)}"


def test_range_allocator_full_release_restores_one_range(driver):
    cmds = ["a 1000", "a 2000", "a 3000", "r 1024", "r 0", "r 3072"]
    out = subprocess.run([driver], input="8192\n" + "\n".join(cmds) + "\n",
                         capture_output=True, text=True, check=True).stdout.split()
    assert out[:6] == ["0", "1024", "3072", "1", "1", "1"]
    assert out[6:9] == ["0", "8192", "1"]


def _gw():
    from paper_2404_08970_amd import gw
    return gw


def test_request_footprint_arithmetic():
    gw = _gw()
    for n, k in [(128, 1), (1000, 2), (4096, 1), (8192, 2)]:
        X = gw.unit_grid((n,), k)
        b = gw.request_bytes(X, X)
        # T and the gradient (16 MN), Sinkhorn partials (12 nb N, nb <= 256)
        rb = (n + 255) // 256
        nb = (n + rb - 1) // rb
        assert b >= 16 * n * n + 12 * nb * n
        assert b <= 24 * n * n + 12 * nb * n + 64 * 1024 * 8
        assert b % 256 == 0
    X2 = gw.unit_grid((96, 96), 1)
    assert gw.request_bytes(X2, X2) >= 16 * 9216 ** 2
    assert gw.request_bytes(gw.unit_grid((10,), 9), gw.unit_grid((10,), 1)) == 0  # k > KMAX


def test_table_bytes():
    gw = _gw()
    assert gw.server_table_bytes(0) == 0
    assert gw.server_table_bytes(5000) == 0
    a, b = gw.server_table_bytes(1), gw.server_table_bytes(64)
    assert 0 < a < b and b % 256 == 0


def test_create_validates_before_any_device_call():
    gw = _gw()
    lib = gw.library()
    h = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 40)  # never dereferenced: validation fails first
    assert lib.gw_server_create(None, 1 << 30, 4, 10, None, ctypes.byref(h)) == gw.GW_EINVAL
    assert lib.gw_server_create(ctypes.c_void_p((1 << 40) + 8), 1 << 30, 4, 10, None,
                                ctypes.byref(h)) == gw.GW_EINVAL          # misaligned
    assert lib.gw_server_create(fake, 1 << 30, 0, 10, None, ctypes.byref(h)) == gw.GW_EINVAL
    assert lib.gw_server_create(fake, 1 << 30, 4, 0, None, ctypes.byref(h)) == gw.GW_EINVAL
    assert lib.gw_server_create(fake, 1 << 30, 4, 1001, None, ctypes.byref(h)) == gw.GW_EINVAL
    assert lib.gw_server_create(fake, 1024, 4, 10, None, ctypes.byref(h)) == gw.GW_ENOMEM
    assert lib.gw_server_create(fake, 1 << 30, 4, 10, None, None) == gw.GW_EINVAL
    assert not h.value


def test_server_calls_reject_null_handle():
    gw = _gw()
    lib = gw.library()
    s = ctypes.c_int32(0)
    rid = ctypes.c_int64(0)
    res = gw.c_result()
    X = gw.unit_grid((16,), 1)
    r = gw.make_request(X, X, None, None, 1e-2, 1, 1)
    assert lib.gw_server_submit(None, ctypes.byref(r), ctypes.byref(rid)) == gw.GW_EINVAL
    assert lib.gw_server_step(None, None, None) == gw.GW_EINVAL
    assert lib.gw_server_set_boost(None, 2) == gw.GW_EINVAL
    assert lib.gw_server_poll(None, 1, ctypes.byref(s)) == gw.GW_EINVAL
    assert lib.gw_server_result(None, 1, ctypes.byref(res)) == gw.GW_EINVAL
    assert lib.gw_server_release(None, 1) == gw.GW_EINVAL
    assert lib.gw_server_destroy(None) == gw.GW_EINVAL


def test_request_validation():
    gw = _gw()
    lib = gw.library()
    X = gw.unit_grid((16,), 1)
    r = gw.make_request(X, X, None, None, 1e-2, 1, 1)
    r.p = r.q = 256
    assert lib.gw_server_request_bytes(ctypes.byref(r)) > 0
    for field, bad in [("eps", 0.0), ("eps", float("nan")), ("outer", -1), ("inner", -1),
                       ("flags", 4), ("reserved", 1), ("p", 0), ("q", 260)]:
        r2 = gw.make_request(X, X, None, None, 1e-2, 1, 1)
        r2.p = r2.q = 256
        setattr(r2, field, bad)
        assert lib.gw_server_request_bytes(ctypes.byref(r2)) == 0, field
    big = gw.unit_grid((16385,), 1)
    r3 = gw.make_request(X, big, None, None, 1e-2, 1, 1)
    r3.p = r3.q = 256
    assert lib.gw_server_request_bytes(ctypes.byref(r3)) == 0   # N > 16384
