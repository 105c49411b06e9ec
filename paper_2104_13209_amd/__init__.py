"""Exact k-clique counting on AMD Instinct MI355X (gfx950).

Thin Python binding over the C ABI of ``libkc.so`` (declared in
``include/kc.h``).  This module only marshals arguments: torch tensors provide
device memory and the current HIP stream; every step of the computation
(orientation, extraction, traversal, reduction) runs in the library's kernels.
The library must be built (``python -m paper_2104_13209_amd._build``); importing
the extension fails loudly if it is missing.

Method: Almasri, El Hajj, Nagi, Xiong, Hwu, "Parallel K-clique Counting on
GPUs" (ICS 2022, arXiv 2104.13209).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libkc.so")

ORDER_DEGREE, ORDER_DEGENERACY = 0, 1
SCHEME_AUTO, SCHEME_VC, SCHEME_EC = 0, 1, 2
OK, EINVAL, ENOMEM, EOVERFLOW, EDEVICE, ECANCELED, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MAX_DMAX = 1024


class KcError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__("%s: %s (status %d)" % (what, strerror(code), code))
        self.code = code


class _U128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p)]


class _Dag(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("d_max", ctypes.c_int32),
                ("degeneracy", ctypes.c_int32), ("order", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("src", ctypes.c_void_p), ("perm", ctypes.c_void_p)]


class Profile(ctypes.Structure):
    """kc_profile: per-phase GPU times (ms) and, with collect_stats, work counters."""
    _fields_ = [("ms_classify", ctypes.c_float), ("ms_light", ctypes.c_float),
                ("ms_heavy", ctypes.c_float), ("ms_total", ctypes.c_float),
                ("nodes", ctypes.c_uint64 * 2), ("word_ops", ctypes.c_uint64 * 2),
                ("light_roots", ctypes.c_int32), ("heavy_roots", ctypes.c_int32)]


class _Opts(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("width", ctypes.c_int32),
                ("collect_stats", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("test_preload", ctypes.c_uint64), ("profile", ctypes.POINTER(Profile))]


_lib = None


def lib():
    """The loaded libkc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libkc.so is not built: run `python -m paper_2104_13209_amd._build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.kc_orient_workspace.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.kc_orient_workspace.restype = ctypes.c_size_t
        L.kc_orient.argtypes = [P(_Csr), ctypes.c_int32, P(_Dag), ctypes.c_void_p, ctypes.c_size_t,
                                ctypes.c_int32, ctypes.c_void_p]
        L.kc_orient.restype = ctypes.c_int32
        L.kc_count_workspace.argtypes = [P(_Dag), ctypes.c_int32, ctypes.c_int32, P(_Opts)]
        L.kc_count_workspace.restype = ctypes.c_size_t
        L.kc_count.argtypes = [P(_Dag), ctypes.c_int32, ctypes.c_int32, P(_U128), ctypes.c_void_p,
                               ctypes.c_size_t, P(_Opts), ctypes.c_void_p]
        L.kc_count.restype = ctypes.c_int32
        L.kc_count_all.argtypes = [P(_Dag), ctypes.c_int32, P(_U128), ctypes.c_int32, P(ctypes.c_int32),
                                   ctypes.c_void_p, ctypes.c_size_t, P(_Opts), ctypes.c_void_p]
        L.kc_count_all.restype = ctypes.c_int32
        L.kc_strerror.argtypes = [ctypes.c_int32]
        L.kc_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().kc_strerror(code).decode()
    except ImportError:
        return "status %d" % code


def _stream_handle(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() > 0 else 0)


@dataclass
class Csr:
    """Undirected graph resident on the device (sorted simple symmetric CSR)."""
    n: int
    row_ptr: torch.Tensor   # int32[n+1]
    col: torch.Tensor       # int32[nnz]

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    def _c(self) -> _Csr:
        return _Csr(self.n, self.nnz, _ptr(self.row_ptr), _ptr(self.col))


@dataclass
class Dag:
    """Oriented graph on the device; vertex i of the DAG is input vertex perm[i]."""
    n: int
    m: int
    d_max: int
    degeneracy: int
    order: int
    row_ptr: torch.Tensor
    col: torch.Tensor
    src: torch.Tensor
    perm: torch.Tensor

    def _c(self) -> _Dag:
        return _Dag(self.n, self.m, self.d_max, self.degeneracy, self.order, _ptr(self.row_ptr),
                    _ptr(self.col), _ptr(self.src), _ptr(self.perm))


def to_device(graph, device="cuda") -> Csr:
    """Copy a host graph (anything with n, row_ptr, col as int arrays) to the device."""
    rp = torch.as_tensor(np.ascontiguousarray(graph.row_ptr, dtype=np.int32)).to(device)
    cl = torch.as_tensor(np.ascontiguousarray(graph.col, dtype=np.int32)).to(device)
    return Csr(int(graph.n), rp, cl)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def orient_workspace_bytes(n: int, nnz: int, order: int) -> int:
    return int(lib().kc_orient_workspace(n, nnz, order))


def orient(g: Csr, order: int = ORDER_DEGREE, validate: bool = True, ws: torch.Tensor | None = None,
           out: Dag | None = None, stream=None) -> Dag:
    """Orient g into a DAG by degree or degeneracy order (kc_orient)."""
    L = lib()
    dev = g.row_ptr.device
    m = g.nnz // 2
    if out is None:
        out = Dag(g.n, m, 0, -1, order,
                  torch.empty(g.n + 1, dtype=torch.int32, device=dev),
                  torch.empty(max(m, 1), dtype=torch.int32, device=dev),
                  torch.empty(max(m, 1), dtype=torch.int32, device=dev),
                  torch.empty(max(g.n, 1), dtype=torch.int32, device=dev))
    need = orient_workspace_bytes(g.n, g.nnz, order)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    cg = g._c()
    cd = out._c()
    st = L.kc_orient(ctypes.byref(cg), order, ctypes.byref(cd), _ptr(ws), ws.numel(), int(bool(validate)),
                     _stream_handle(stream))
    if st != OK:
        raise KcError(st, "kc_orient")
    out.n, out.m, out.d_max, out.degeneracy, out.order = cd.n, cd.m, cd.d_max, cd.degeneracy, cd.order
    return out


def _opts(scheme: int, width: int, test_preload: int, profile: Profile | None = None,
          collect_stats: bool = False) -> _Opts:
    o = _Opts(scheme, width, int(bool(collect_stats)), 0, test_preload, None)
    if profile is not None:
        o.profile = ctypes.pointer(profile)
    return o


def count_workspace_bytes(d: Dag, k: int, pivot: bool, scheme: int = 0, width: int = 0) -> int:
    cd = d._c()
    o = _opts(scheme, width, 0)
    return int(lib().kc_count_workspace(ctypes.byref(cd), k, int(bool(pivot)), ctypes.byref(o)))


def count_status(d: Dag, k: int, pivot: bool = False, scheme: int = SCHEME_AUTO, width: int = 0,
                 ws: torch.Tensor | None = None, test_preload: int = 0, stream=None,
                 profile: Profile | None = None, collect_stats: bool = False):
    """(status, count) of kc_count without raising."""
    L = lib()
    cd = d._c()
    o = _opts(scheme, width, test_preload, profile, collect_stats)
    need = int(L.kc_count_workspace(ctypes.byref(cd), k, int(bool(pivot)), ctypes.byref(o)))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, d.row_ptr.device)
    res = _U128(0, 0)
    st = L.kc_count(ctypes.byref(cd), k, int(bool(pivot)), ctypes.byref(res), _ptr(ws), ws.numel(),
                    ctypes.byref(o), _stream_handle(stream))
    return st, int(res.lo) | (int(res.hi) << 64)


def count(d: Dag, k: int, pivot: bool = False, scheme: int = SCHEME_AUTO, width: int = 0,
          ws: torch.Tensor | None = None, stream=None, profile: Profile | None = None,
          collect_stats: bool = False) -> int:
    """Number of k-cliques (kc_count); exact Python int."""
    st, val = count_status(d, k, pivot, scheme, width, ws, 0, stream, profile, collect_stats)
    if st != OK:
        raise KcError(st, "kc_count")
    return val


def count_all(d: Dag, pivot: bool = True, cap: int | None = None, scheme: int = SCHEME_AUTO,
              width: int = 0, ws: torch.Tensor | None = None, stream=None,
              profile: Profile | None = None):
    """([c_0, ..., c_cap], omega) for every clique size (kc_count_all)."""
    L = lib()
    if cap is None:
        cap = d.d_max + 2
    cap = max(int(cap), 2)
    cd = d._c()
    o = _opts(scheme, width, 0, profile)
    need = int(L.kc_count_workspace(ctypes.byref(cd), 0, int(bool(pivot)), ctypes.byref(o)))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, d.row_ptr.device)
    res = (_U128 * (cap + 1))()
    om = ctypes.c_int32(0)
    st = L.kc_count_all(ctypes.byref(cd), int(bool(pivot)), res, cap, ctypes.byref(om), _ptr(ws),
                        ws.numel(), ctypes.byref(o), _stream_handle(stream))
    if st != OK:
        raise KcError(st, "kc_count_all")
    return [int(r.lo) | (int(r.hi) << 64) for r in res], int(om.value)


def dag_to_host(d: Dag):
    """(row_ptr, col, src, perm) as numpy arrays."""
    m = d.m
    return (d.row_ptr.cpu().numpy(), d.col[:m].cpu().numpy(), d.src[:m].cpu().numpy(),
            d.perm[:d.n].cpu().numpy())
