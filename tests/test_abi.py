"""The C-ABI library loads and exports every symbol include/kc.h declares; host-only
argument checks behave as documented.  No device work happens here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kc.h")
LIB = os.path.join(ROOT, "paper_2104_13209_amd", "libkc.so")


def declared():
    text = open(HEADER).read()
    return re.findall(r"KC_API\s+[\w\s\*]+?\b(kc_\w+)\s*\(", text)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libkc.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = declared()
    for want in ("kc_orient", "kc_orient_workspace", "kc_count", "kc_count_workspace",
                 "kc_count_all", "kc_count_noalloc", "kc_strerror"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared():
        assert hasattr(lib, name), name


def test_host_side_argument_checks(lib):
    import paper_2104_13209_amd as kc
    L = kc.lib()
    assert L.kc_strerror(0) == b"ok"
    assert L.kc_strerror(-3).startswith(b"count exceeds")
    assert L.kc_orient_workspace(-1, 0, 0) == 0
    a = L.kc_orient_workspace(1000, 10000, 0)
    b = L.kc_orient_workspace(100000, 1000000, 1)
    assert 0 < a < b
    # argument errors are reported before any device call
    res = kc._U128(0, 0)
    dag = kc._Dag(10, 20, 5, -1, 0, ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.c_void_p(1))
    assert L.kc_count(ctypes.byref(dag), 0, 0, ctypes.byref(res), None, 0, None, None) == kc.EINVAL
    assert L.kc_count(None, 3, 0, ctypes.byref(res), None, 0, None, None) == kc.EINVAL
    assert L.kc_count(ctypes.byref(dag), 1, 0, ctypes.byref(res), None, 0, None, None) == kc.OK
    assert (res.lo, res.hi) == (10, 0)
    assert L.kc_count(ctypes.byref(dag), 2, 1, ctypes.byref(res), None, 0, None, None) == kc.OK
    assert (res.lo, res.hi) == (20, 0)
    # a workspace that is too small is refused
    assert L.kc_count(ctypes.byref(dag), 4, 0, ctypes.byref(res), ctypes.c_void_p(1), 1, None, None) == kc.ENOMEM
    assert L.kc_orient(None, 0, None, None, 0, 1, None) == kc.EINVAL
    # every order is accepted (a missing workspace is the next error), anything
    # else is refused, all before any device call
    g10 = kc._Csr(10, 20, ctypes.c_void_p(1), ctypes.c_void_p(1))
    for order in (kc.ORDER_DEGREE, kc.ORDER_DEGENERACY, kc.ORDER_APPROX_DEGENERACY, kc.ORDER_COLOR):
        assert L.kc_orient(ctypes.byref(g10), order, ctypes.byref(dag), None, 0, 1, None) == kc.ENOMEM, order
    for order in (-1, 4):
        assert L.kc_orient(ctypes.byref(g10), order, ctypes.byref(dag), None, 0, 1, None) == kc.EINVAL, order
    # kc_count_noalloc refuses a DAG whose workspace exceeds its fixed scratch
    # before touching the device
    big = kc._Dag(5_000_000, 5_000_000, 64, -1, 0, ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.c_void_p(1),
                  ctypes.c_void_p(1))
    assert L.kc_count_workspace(ctypes.byref(big), 4, 0, None) > 64 << 20
    assert L.kc_count_noalloc(ctypes.byref(big), 4, 0, ctypes.byref(res), None, None) == kc.ENOMEM
    assert L.kc_count_noalloc(ctypes.byref(big), 1, 0, ctypes.byref(res), None, None) == kc.OK
    assert (res.lo, res.hi) == (5_000_000, 0)
    # out-degrees past the wide-root limit are refused before any device call;
    # per-vertex counts stay within the on-chip limit
    p1 = ctypes.c_void_p(1)
    over = kc._Dag(20_000, 40_000, kc.MAX_DMAX_WIDE + 1, -1, 0, p1, p1, p1, p1)
    wide = kc._Dag(20_000, 40_000, 2 * kc.MAX_DMAX, -1, 0, p1, p1, p1, p1)
    chip = kc._Dag(20_000, 40_000, kc.MAX_DMAX, -1, 0, p1, p1, p1, p1)
    for pivot in (0, 1):
        assert L.kc_count(ctypes.byref(over), 4, pivot, ctypes.byref(res), p1, 1 << 40, None, None) == kc.EUNSUPPORTED
    counts = (kc._U128 * 8)()
    om = ctypes.c_int32(0)
    assert L.kc_count_all(ctypes.byref(over), 1, counts, 7, ctypes.byref(om), p1, 1 << 40, None, None) == \
        kc.EUNSUPPORTED
    assert L.kc_count_local(ctypes.byref(wide), 4, 0, p1, p1, 1 << 40, None, None) == kc.EUNSUPPORTED
    # wide roots add their global-memory slabs to the workspace
    assert L.kc_count_workspace(ctypes.byref(wide), 4, 0, None) > L.kc_count_workspace(ctypes.byref(chip), 4, 0, None)


def test_product_path_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_2104_13209_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", text, re.M), f
                assert "kc_oracle" not in text and "liboracle" not in text, f
