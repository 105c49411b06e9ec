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

import atexit
import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libkc.so")

ORDER_DEGREE, ORDER_DEGENERACY, ORDER_APPROX_DEGENERACY, ORDER_COLOR = 0, 1, 2, 3
SCHEME_AUTO, SCHEME_VC, SCHEME_EC = 0, 1, 2
OPT_NO_HANDOFF, OPT_SINGLE_STREAM, OPT_NO_BITSETS = 1, 2, 4
OK, EINVAL, ENOMEM, EOVERFLOW, EDEVICE, ECANCELED, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MAX_DMAX = 1024          # out-degree whose roots keep their bitset rows on chip
MAX_DMAX_WIDE = 8192     # out-degree limit of kc_count / kc_count_all (wide roots in global memory)


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
                ("light_roots", ctypes.c_int32), ("heavy_roots", ctypes.c_int32),
                ("ms_width", ctypes.c_float * 6), ("roots_width", ctypes.c_int32 * 6),
                ("nodes_width", ctypes.c_uint64 * 6), ("words_width", ctypes.c_uint64 * 6),
                ("iters_width", ctypes.c_uint64 * 6), ("expand_width", ctypes.c_uint64 * 6),
                ("waves_width", ctypes.c_int32 * 6),
                ("busy_width", ctypes.c_float * 6), ("items_width", ctypes.c_int32 * 6),
                ("cwords_width", ctypes.c_uint64 * 6)]


class _Opts(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("width", ctypes.c_int32),
                ("collect_stats", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("test_preload", ctypes.c_uint64), ("profile", ctypes.POINTER(Profile)),
                ("cancel", ctypes.c_void_p), ("handoff_after", ctypes.c_int32),
                ("handoff_every", ctypes.c_int32)]


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
        L.kc_count_noalloc.argtypes = [P(_Dag), ctypes.c_int32, ctypes.c_int32, P(_U128), P(_Opts),
                                       ctypes.c_void_p]
        L.kc_count_noalloc.restype = ctypes.c_int32
        L.kc_strerror.argtypes = [ctypes.c_int32]
        L.kc_strerror.restype = ctypes.c_char_p
        L.kc_count_local.argtypes = [P(_Dag), ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_size_t, P(_Opts), ctypes.c_void_p]
        L.kc_count_local.restype = ctypes.c_int32
        L.kc_list.argtypes = [P(_Dag), ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, P(ctypes.c_uint64),
                              ctypes.c_void_p, ctypes.c_size_t, P(_Opts), ctypes.c_void_p]
        L.kc_list.restype = ctypes.c_int32
        L.kc_shutdown.argtypes = []
        L.kc_shutdown.restype = None
        # release pooled streams and events while the HIP runtime is alive
        atexit.register(L.kc_shutdown)
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
    """Orient g into a DAG by degree, degeneracy, approximate degeneracy or
    colouring order (kc_orient)."""
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
          collect_stats: bool = False, handoff: bool = True, single_stream: bool = False,
          cancel: int = 0, handoff_after: int = 0, handoff_every: int = 0, bitsets: bool = True) -> _Opts:
    flags = ((0 if handoff else OPT_NO_HANDOFF) | (OPT_SINGLE_STREAM if single_stream else 0) |
             (0 if bitsets else OPT_NO_BITSETS))
    o = _Opts(scheme, width, int(bool(collect_stats)), flags, test_preload, None,
              ctypes.c_void_p(cancel or None), handoff_after, handoff_every)
    if profile is not None:
        o.profile = ctypes.pointer(profile)
    return o


def count_workspace_bytes(d: Dag, k: int, pivot: bool, scheme: int = 0, width: int = 0) -> int:
    cd = d._c()
    o = _opts(scheme, width, 0)
    return int(lib().kc_count_workspace(ctypes.byref(cd), k, int(bool(pivot)), ctypes.byref(o)))


def count_status(d: Dag, k: int, pivot: bool = False, scheme: int = SCHEME_AUTO, width: int = 0,
                 ws: torch.Tensor | None = None, test_preload: int = 0, stream=None,
                 profile: Profile | None = None, collect_stats: bool = False, handoff: bool = True,
                 single_stream: bool = False, cancel: int = 0, handoff_after: int = 0,
                 handoff_every: int = 0, bitsets: bool = True):
    """(status, count) of kc_count without raising.  cancel: address of a
    device-readable int32 (device memory or mapped host memory) that stops the
    count with ECANCELED once it holds a non-zero value."""
    L = lib()
    cd = d._c()
    o = _opts(scheme, width, test_preload, profile, collect_stats, handoff, single_stream, cancel,
              handoff_after, handoff_every, bitsets)
    need = int(L.kc_count_workspace(ctypes.byref(cd), k, int(bool(pivot)), ctypes.byref(o)))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, d.row_ptr.device)
    res = _U128(0, 0)
    st = L.kc_count(ctypes.byref(cd), k, int(bool(pivot)), ctypes.byref(res), _ptr(ws), ws.numel(),
                    ctypes.byref(o), _stream_handle(stream))
    return st, int(res.lo) | (int(res.hi) << 64)


def count(d: Dag, k: int, pivot: bool = False, scheme: int = SCHEME_AUTO, width: int = 0,
          ws: torch.Tensor | None = None, stream=None, profile: Profile | None = None,
          collect_stats: bool = False, handoff: bool = True, single_stream: bool = False,
          handoff_after: int = 0, handoff_every: int = 0, bitsets: bool = True) -> int:
    """Number of k-cliques (kc_count); exact Python int.  handoff=False keeps
    every subtree on the wavefront that found it; single_stream=True keeps every
    launch on `stream` (KC_OPT_* flags); handoff_after / handoff_every lower the
    handoff thresholds (0 = defaults); bitsets=False runs the list-intersection
    ablation (KC_OPT_NO_BITSETS)."""
    st, val = count_status(d, k, pivot, scheme, width, ws, 0, stream, profile, collect_stats, handoff,
                           single_stream, 0, handoff_after, handoff_every, bitsets)
    if st != OK:
        raise KcError(st, "kc_count")
    return val


def count_all_status(d: Dag, pivot: bool = True, cap: int | None = None, scheme: int = SCHEME_AUTO,
                     width: int = 0, ws: torch.Tensor | None = None, stream=None,
                     profile: Profile | None = None, cancel: int = 0, collect_stats: bool = False,
                     handoff: bool = True, handoff_after: int = 0, handoff_every: int = 0):
    """(status, [c_0, ..., c_cap], omega) of kc_count_all without raising."""
    L = lib()
    if cap is None:
        cap = d.d_max + 2
    cap = max(int(cap), 2)
    cd = d._c()
    o = _opts(scheme, width, 0, profile, collect_stats, handoff=handoff, cancel=cancel,
              handoff_after=handoff_after, handoff_every=handoff_every)
    need = int(L.kc_count_workspace(ctypes.byref(cd), 0, int(bool(pivot)), ctypes.byref(o)))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, d.row_ptr.device)
    res = (_U128 * (cap + 1))()
    om = ctypes.c_int32(0)
    st = L.kc_count_all(ctypes.byref(cd), int(bool(pivot)), res, cap, ctypes.byref(om), _ptr(ws),
                        ws.numel(), ctypes.byref(o), _stream_handle(stream))
    return st, [int(r.lo) | (int(r.hi) << 64) for r in res], int(om.value)


def count_all(d: Dag, pivot: bool = True, cap: int | None = None, scheme: int = SCHEME_AUTO,
              width: int = 0, ws: torch.Tensor | None = None, stream=None,
              profile: Profile | None = None, collect_stats: bool = False):
    """([c_0, ..., c_cap], omega) for every clique size (kc_count_all)."""
    st, counts, om = count_all_status(d, pivot, cap, scheme, width, ws, stream, profile,
                                      collect_stats=collect_stats)
    if st != OK:
        raise KcError(st, "kc_count_all")
    return counts, om


def count_local(d: Dag, k: int, pivot: bool = False, scheme: int = SCHEME_AUTO,
                ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Per-vertex k-clique counts (kc_count_local): an int64 tensor of n entries
    indexed by input vertex id, holding the unsigned 64-bit counts."""
    L = lib()
    cd = d._c()
    o = _opts(scheme, 0, 0)
    need = int(L.kc_count_workspace(ctypes.byref(cd), k, int(bool(pivot)), ctypes.byref(o)))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, d.row_ptr.device)
    out = torch.empty(max(d.n, 1), dtype=torch.int64, device=d.row_ptr.device)
    st = L.kc_count_local(ctypes.byref(cd), k, int(bool(pivot)), _ptr(out), _ptr(ws), ws.numel(), ctypes.byref(o),
                          _stream_handle(stream))
    if st != OK:
        raise KcError(st, "kc_count_local")
    return out[:d.n]


def list_cliques_status(d: Dag, k: int, cap: int, scheme: int = SCHEME_AUTO, ws: torch.Tensor | None = None,
                        stream=None, cancel: int = 0):
    """(status, total, rows) of kc_list without raising: rows is an int32 tensor
    of min(total, cap) cliques (k input ids each, ascending orientation rank)."""
    L = lib()
    cd = d._c()
    o = _opts(scheme, 0, 0, cancel=cancel)
    need = int(L.kc_count_workspace(ctypes.byref(cd), k, 0, ctypes.byref(o)))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, d.row_ptr.device)
    cap = max(int(cap), 0)
    out = torch.empty((max(cap, 1), max(k, 1)), dtype=torch.int32, device=d.row_ptr.device)
    total = ctypes.c_uint64(0)
    st = L.kc_list(ctypes.byref(cd), k, _ptr(out), cap, ctypes.byref(total), _ptr(ws), ws.numel(), ctypes.byref(o),
                   _stream_handle(stream))
    t = int(total.value)
    return st, t, out[:min(t, cap)]


def list_cliques(d: Dag, k: int, cap: int | None = None, scheme: int = SCHEME_AUTO, ws: torch.Tensor | None = None,
                 stream=None):
    """(total, rows): the k-cliques of the DAG's graph (kc_list).  Without a cap
    the output is sized by a count first, so every clique is listed."""
    if cap is None:
        cap = count(d, k, pivot=True, scheme=scheme) if k >= 3 else (d.n if k == 1 else d.m)
    st, total, rows = list_cliques_status(d, k, cap, scheme, ws, stream)
    if st != OK:
        raise KcError(st, "kc_list")
    return total, rows


def count_noalloc_status(d: Dag, k: int, pivot: bool = False, scheme: int = SCHEME_AUTO, stream=None):
    """(status, count) of kc_count_noalloc: kc_count on the library's fixed
    device scratch instead of a caller workspace (no allocation anywhere)."""
    cd = d._c()
    o = _opts(scheme, 0, 0)
    res = _U128(0, 0)
    st = lib().kc_count_noalloc(ctypes.byref(cd), k, int(bool(pivot)), ctypes.byref(res), ctypes.byref(o),
                                _stream_handle(stream))
    return st, int(res.lo) | (int(res.hi) << 64)


def count_noalloc(d: Dag, k: int, pivot: bool = False, scheme: int = SCHEME_AUTO, stream=None) -> int:
    st, val = count_noalloc_status(d, k, pivot, scheme, stream)
    if st != OK:
        raise KcError(st, "kc_count_noalloc")
    return val


def dag_to_host(d: Dag):
    """(row_ptr, col, src, perm) as numpy arrays."""
    m = d.m
    return (d.row_ptr.cpu().numpy(), d.col[:m].cpu().numpy(), d.src[:m].cpu().numpy(),
            d.perm[:d.n].cpu().numpy())


# ---------------------------------------------------------------- batched

MAX_BUCKETS = 8


class _Batch(ctypes.Structure):
    _fields_ = [("ngraphs", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int32),
                ("max_degree", ctypes.c_int32), ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("voff", ctypes.c_void_p), ("max_graph_edges", ctypes.c_int32)]


class BatchPlan(ctypes.Structure):
    """kc_batch_plan: root scheme and traversal width per graph-size bucket
    (n <= n_hi[b]); width 0 = lane walk, 2..32 = sub-wavefront groups."""
    _fields_ = [("nbuckets", ctypes.c_int32), ("n_hi", ctypes.c_int32 * MAX_BUCKETS),
                ("scheme", ctypes.c_int32 * MAX_BUCKETS), ("width", ctypes.c_int32 * MAX_BUCKETS)]

    @classmethod
    def make(cls, buckets):
        """buckets: list of (n_hi, scheme) or (n_hi, scheme, width) in ascending n_hi."""
        p = cls()
        p.nbuckets = len(buckets)
        for i, b in enumerate(buckets):
            p.n_hi[i] = int(b[0])
            p.scheme[i] = int(b[1])
            p.width[i] = int(b[2]) if len(b) > 2 else 0
        return p

    def as_list(self):
        return [(int(self.n_hi[i]), int(self.scheme[i]), int(self.width[i])) for i in range(self.nbuckets)]


@dataclass
class BatchDev:
    """Packed independent graphs resident on the device."""
    ngraphs: int
    n: int
    max_degree: int
    row_ptr: torch.Tensor
    col: torch.Tensor
    voff: torch.Tensor
    max_graph_edges: int = 0

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    def _c(self) -> _Batch:
        return _Batch(self.ngraphs, self.n, self.nnz, self.max_degree, _ptr(self.row_ptr), _ptr(self.col),
                      _ptr(self.voff), self.max_graph_edges)


def batch_to_device(b, device="cuda") -> BatchDev:
    """Copy a host batch (voff, row_ptr, col arrays) to the device."""
    rp = np.asarray(b.row_ptr, dtype=np.int64)
    deg = np.diff(rp)
    ends = rp[np.asarray(b.voff, dtype=np.int64)]
    max_m = int(np.diff(ends).max() // 2) if ends.size > 1 else 0
    return BatchDev(int(b.voff.shape[0] - 1), int(b.voff[-1]), int(deg.max()) if deg.size else 0,
                    torch.as_tensor(np.ascontiguousarray(b.row_ptr, np.int32)).to(device),
                    torch.as_tensor(np.ascontiguousarray(b.col, np.int32)).to(device),
                    torch.as_tensor(np.ascontiguousarray(b.voff, np.int32)).to(device), max_m)


def _batch_lib():
    L = lib()
    if not getattr(L, "_batch_ready", False):
        L.kc_batch_workspace.argtypes = [ctypes.POINTER(_Batch), ctypes.c_int32]
        L.kc_batch_workspace.restype = ctypes.c_size_t
        L.kc_batch_count.argtypes = [ctypes.POINTER(_Batch), ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_size_t, ctypes.POINTER(BatchPlan), ctypes.c_void_p]
        L.kc_batch_count.restype = ctypes.c_int32
        L._batch_ready = True
    return L


def batch_workspace_bytes(b: BatchDev, k: int) -> int:
    cb = b._c()
    return int(_batch_lib().kc_batch_workspace(ctypes.byref(cb), k))


def batch_count_async(b: BatchDev, k: int, out: torch.Tensor, ws: torch.Tensor, plan: BatchPlan | None = None,
                      stream=None) -> None:
    """Enqueue kc_batch_count: per-graph counts into out (int64 [2*ngraphs] holding
    unsigned {lo, hi} pairs).  No synchronisation: capturable in a HIP graph."""
    L = _batch_lib()
    cb = b._c()
    st = L.kc_batch_count(ctypes.byref(cb), k, _ptr(out), _ptr(ws), ws.numel(),
                          ctypes.byref(plan) if plan is not None else None, _stream_handle(stream))
    if st != OK:
        raise KcError(st, "kc_batch_count")


def counts_from_device(out: torch.Tensor):
    """Exact per-graph counts (Python ints) from the {lo, hi} pairs."""
    a = out.cpu().numpy().view(np.uint64).reshape(-1, 2)
    return [int(lo) | (int(hi) << 64) for lo, hi in a]


def batch_count(b: BatchDev, k: int, plan: BatchPlan | None = None):
    """Per-graph k-clique counts of a batch (eager call + copy back)."""
    ws = _workspace(batch_workspace_bytes(b, k), b.row_ptr.device)
    out = torch.empty(2 * b.ngraphs, dtype=torch.int64, device=b.row_ptr.device)
    batch_count_async(b, k, out, ws, plan)
    torch.cuda.synchronize()
    return counts_from_device(out)


class BatchGraph:
    """kc_batch_count captured once in a HIP graph (torch.cuda.CUDAGraph) and replayed."""

    def __init__(self, b: BatchDev, k: int, plan: BatchPlan | None = None):
        self.b, self.k, self.plan = b, k, plan
        dev = b.row_ptr.device
        self.ws = _workspace(batch_workspace_bytes(b, k), dev)
        self.out = torch.empty(2 * b.ngraphs, dtype=torch.int64, device=dev)
        # one eager call first (loads kernels, sets attributes), then capture
        batch_count_async(b, k, self.out, self.ws, plan)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(self.graph, stream=side):
                batch_count_async(b, k, self.out, self.ws, plan, stream=side)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()

    def replay(self):
        self.graph.replay()

    def counts(self):
        torch.cuda.synchronize()
        return counts_from_device(self.out)


# ---------------------------------------------------------------- serving

class QueryResult(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("graph", ctypes.c_int32), ("k", ctypes.c_int32),
                ("pivot", ctypes.c_int32), ("status", ctypes.c_int32), ("count", _U128),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("workspace", ctypes.c_uint64), ("lds", ctypes.c_uint64)]

    @property
    def value(self) -> int:
        return int(self.count.lo) | (int(self.count.hi) << 64)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit


def _server_lib():
    L = lib()
    if not getattr(L, "_server_ready", False):
        L.kc_server_create.argtypes = [ctypes.POINTER(_Dag), ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                       ctypes.POINTER(ctypes.c_void_p)]
        L.kc_server_create.restype = ctypes.c_int32
        L.kc_server_submit.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_uint64)]
        L.kc_server_submit.restype = ctypes.c_int32
        L.kc_server_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(QueryResult)]
        L.kc_server_wait.restype = ctypes.c_int32
        L.kc_server_destroy.argtypes = [ctypes.c_void_p]
        L.kc_server_destroy.restype = ctypes.c_int32
        L._server_ready = True
    return L


class Server:
    """kc_server: continuous batching of count queries over resident DAGs."""

    def __init__(self, dags, slots: int = 4, mem_budget: int = 8 << 30):
        L = _server_lib()
        self._dags = list(dags)          # keep the device tensors alive
        arr = (_Dag * len(self._dags))(*[d._c() for d in self._dags])
        self._arr = arr
        h = ctypes.c_void_p()
        st = L.kc_server_create(arr, len(self._dags), slots, mem_budget, ctypes.byref(h))
        if st != OK:
            raise KcError(st, "kc_server_create")
        self._h = h

    def submit(self, graph: int, k: int, pivot: bool = False) -> int:
        t = ctypes.c_uint64(0)
        st = _server_lib().kc_server_submit(self._h, graph, k, int(bool(pivot)), ctypes.byref(t))
        if st != OK:
            raise KcError(st, "kc_server_submit")
        return int(t.value)

    def wait(self, ticket: int) -> QueryResult:
        r = QueryResult()
        st = _server_lib().kc_server_wait(self._h, ticket, ctypes.byref(r))
        if st != OK:
            raise KcError(st, "kc_server_wait")
        return r

    def close(self):
        if self._h:
            _server_lib().kc_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def replay_trace(server: Server, trace, progress=None):
    """Submit (t_arrival_s, graph, k, pivot) queries at their arrival offsets from
    now (open loop) and return the results in submission order.  progress, if
    given, is called with the number of results collected every 25 results."""
    import time
    t0 = time.perf_counter()
    tickets = []
    for t_arr, g, k, piv in trace:
        while True:
            dt = t_arr - (time.perf_counter() - t0)
            if dt <= 0:
                break
            time.sleep(min(dt, 0.002) if dt > 0.0005 else 0)
        tickets.append(server.submit(g, k, piv))
    out = []
    for t in tickets:
        out.append(server.wait(t))
        if progress is not None and len(out) % 25 == 0:
            progress(len(out))
    return out
