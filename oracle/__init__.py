"""CPU oracle for exact k-clique counting -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never loads it and shares no code with it.

``kc_oracle.c`` is a plain, single-threaded counter written from the paper
(orientation of Sec. 3.1; depth-first walks of the orientation tree of Sec. 2.2
and the pivoting tree of Sec. 2.3), in unsigned 128-bit integer arithmetic.
``kc_brute.c`` is an independent brute-force enumerator for graphs of at most 64
vertices.  This module compiles both with gcc and wraps them with ctypes over
numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "kc_oracle.c"), os.path.join(_HERE, "kc_brute.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

DEGREE, DEGENERACY, APPROX_DEGENERACY, COLOR = 0, 1, 2, 3
VC, EC = 1, 2
OK, EINVAL, ENOMEM, EOVERFLOW = 0, -1, -2, -3


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__("%s failed with code %d" % (what, code))
        self.code = code


def build(force: bool = False) -> str:
    newest = max(os.path.getmtime(s) for s in _SRCS)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=gnu11", "-Wall",
                               "-o", tmp] + _SRCS)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i32 = ctypes.c_int32
        lib.kco_validate.argtypes = [i32, i32p, i32p]
        lib.kco_orient.argtypes = [i32, i32p, i32p, ctypes.c_int, i32p, i32p, i32p, i32p, i32p]
        lib.kco_count.argtypes = [i32, i32p, i32p, i32p, i32p, i32, i32, ctypes.c_int, ctypes.c_int,
                                  i64p, ctypes.c_int64, u64p, u64p, u64p]
        lib.kco_count_all.argtypes = [i32, i32p, i32p, i32p, i32p, i32, ctypes.c_int, ctypes.c_int,
                                      i32, u64p, i32p]
        lib.kco_count_local.argtypes = [i32, i32p, i32p, i32p, i32p, i32, i32, ctypes.c_int,
                                        ctypes.c_int, u64p]
        lib.kco_brute_counts.argtypes = [i32, i32p, i32p, i32, u64p]
        lib.kco_colour.argtypes = [i32, i32p, i32p, i32p]
        lib.kco_splitmix64.argtypes = [ctypes.c_uint64]
        lib.kco_splitmix64.restype = ctypes.c_uint64
        for f in (lib.kco_validate, lib.kco_orient, lib.kco_count, lib.kco_count_all,
                  lib.kco_count_local, lib.kco_brute_counts, lib.kco_colour):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a, t=ctypes.c_int32):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _u128(lo: int, hi: int) -> int:
    return int(lo) | (int(hi) << 64)


@dataclass
class Dag:
    """Oriented graph in ORIGINAL vertex ids: out-lists sorted by id."""
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    rank: np.ndarray
    d_max: int
    degeneracy: int
    # the undirected graph it came from (pivoting levels use it)
    und_row_ptr: np.ndarray
    und_col: np.ndarray

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def out_degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def validate(g) -> bool:
    lib = _load()
    rp, cl = _i32(g.row_ptr), _i32(g.col)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    return lib.kco_validate(g.n, _p(rp), _p(cl)) == OK


def orient(g, order: int = DEGREE) -> Dag:
    lib = _load()
    n = g.n
    rp, cl = _i32(g.row_ptr), _i32(g.col)
    m = cl.shape[0] // 2
    out_ptr = np.zeros(n + 1, dtype=np.int32)
    out_col = np.zeros(max(m, 1), dtype=np.int32)
    rank = np.zeros(max(n, 1), dtype=np.int32)
    dmax = ctypes.c_int32(0)
    degen = ctypes.c_int32(0)
    clp = cl if cl.size else np.zeros(1, dtype=np.int32)
    st = lib.kco_orient(n, _p(rp), _p(clp), order, _p(out_ptr), _p(out_col), _p(rank),
                        ctypes.byref(dmax), ctypes.byref(degen))
    if st != OK:
        raise OracleError(st, "orient")
    return Dag(n, out_ptr, out_col[:m], rank[:n], dmax.value, degen.value, rp, cl)


def splitmix64(x: int) -> int:
    """SplitMix64's output for counter value x (the colouring priority)."""
    return int(_load().kco_splitmix64(x & ((1 << 64) - 1)))


def colour(g) -> np.ndarray:
    """Greedy first-fit colouring in decreasing (priority, id) order."""
    lib = _load()
    rp, cl = _i32(g.row_ptr), _i32(g.col)
    clp = cl if cl.size else np.zeros(1, dtype=np.int32)
    out = np.zeros(max(g.n, 1), dtype=np.int32)
    st = lib.kco_colour(g.n, _p(rp), _p(clp), _p(out))
    if st != OK:
        raise OracleError(st, "colour")
    return out[:g.n]


def _dag_args(d: Dag):
    col = d.col if d.col.size else np.zeros(1, dtype=np.int32)
    ucol = d.und_col if d.und_col.size else np.zeros(1, dtype=np.int32)
    return col, ucol


def count(d: Dag, k: int, pivot: bool = False, scheme: int = VC, roots=None,
          with_nodes: bool = False):
    """c_k of the oriented graph (exact Python int).  `roots` restricts the count to
    those roots (vertex ids for VC, DAG edge indices for EC)."""
    lib = _load()
    col, ucol = _dag_args(d)
    lo, hi, nodes = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint64(0)
    if roots is not None:
        r = np.ascontiguousarray(roots, dtype=np.int64)
        rp_, nr = (_p(r, ctypes.c_int64) if r.size else None), int(r.size)
        if nr == 0:
            return (0, 0) if with_nodes else 0
    else:
        rp_, nr = None, 0
    st = lib.kco_count(d.n, _p(d.row_ptr), _p(col), _p(d.und_row_ptr), _p(ucol), d.d_max, k,
                       int(bool(pivot)), scheme, rp_, nr, ctypes.byref(lo), ctypes.byref(hi),
                       ctypes.byref(nodes))
    if st != OK:
        raise OracleError(st, "count")
    val = _u128(lo.value, hi.value)
    return (val, int(nodes.value)) if with_nodes else val


def count_all(d: Dag, pivot: bool = True, scheme: int = VC, cap: int | None = None):
    """[c_0, c_1, ..., c_cap] (exact ints) and the clique number omega."""
    lib = _load()
    col, ucol = _dag_args(d)
    if cap is None:
        cap = d.d_max + 2
    cap = max(cap, 2)
    buf = np.zeros(2 * (cap + 1), dtype=np.uint64)
    om = ctypes.c_int32(0)
    st = lib.kco_count_all(d.n, _p(d.row_ptr), _p(col), _p(d.und_row_ptr), _p(ucol), d.d_max,
                           int(bool(pivot)), scheme, cap, _p(buf, ctypes.c_uint64), ctypes.byref(om))
    if st != OK:
        raise OracleError(st, "count_all")
    return [_u128(buf[2 * j], buf[2 * j + 1]) for j in range(cap + 1)], om.value


def count_local(d: Dag, k: int, pivot: bool = False, scheme: int = VC):
    """Per-vertex k-clique counts (list of exact ints, original ids)."""
    lib = _load()
    col, ucol = _dag_args(d)
    buf = np.zeros(2 * max(d.n, 1), dtype=np.uint64)
    st = lib.kco_count_local(d.n, _p(d.row_ptr), _p(col), _p(d.und_row_ptr), _p(ucol), d.d_max,
                             k, int(bool(pivot)), scheme, _p(buf, ctypes.c_uint64))
    if st != OK:
        raise OracleError(st, "count_local")
    return [_u128(buf[2 * v], buf[2 * v + 1]) for v in range(d.n)]


def brute_counts(g):
    """Brute-force clique counts [c_0..c_n] for n <= 64 (independent enumerator)."""
    lib = _load()
    if g.n > 64:
        raise ValueError("brute force is limited to 64 vertices")
    rp, cl = _i32(g.row_ptr), _i32(g.col)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    buf = np.zeros(2 * (g.n + 1), dtype=np.uint64)
    st = lib.kco_brute_counts(g.n, _p(rp), _p(cl), g.n, _p(buf, ctypes.c_uint64))
    if st != OK:
        raise OracleError(st, "brute")
    return [_u128(buf[2 * j], buf[2 * j + 1]) for j in range(g.n + 1)]
