"""Seeded synthetic graphs in canonical CSR form.

Shared input source for the CPU oracle's tests and for the GPU path's tests and
benchmark.  Nothing here counts cliques or orients graphs: it only draws graphs
and writes them as a sorted, simple, symmetric CSR (``row_ptr`` int32[n+1],
``col`` int32[2m]), the input format of the paper's Section 3.1.

Random draws come from ``gen.c`` (SplitMix64 streams keyed by seed and index),
so a graph depends only on its parameters and seed.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile gen.c into libsynth.so with gcc (seconds)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        i32p = P(ctypes.c_int32)
        lib.synth_er.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, P(i32p)]
        lib.synth_er.restype = ctypes.c_int64
        lib.synth_chung_lu.argtypes = [ctypes.c_int32, P(ctypes.c_double), ctypes.c_uint64, P(i32p)]
        lib.synth_chung_lu.restype = ctypes.c_int64
        lib.synth_communities.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                                          i32p, P(i32p)]
        lib.synth_communities.restype = ctypes.c_int64
        lib.synth_powerlaw_weights.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_uint64, P(ctypes.c_double)]
        lib.synth_powerlaw_weights.restype = None
        lib.synth_permutation.argtypes = [ctypes.c_int32, ctypes.c_uint64, i32p]
        lib.synth_permutation.restype = None
        lib.synth_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_uniform.restype = ctypes.c_double
        lib.synth_batch.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, i32p,
                                    P(ctypes.c_int64), P(i32p)]
        lib.synth_batch.restype = ctypes.c_int64
        lib.synth_batch_vertices.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_double, ctypes.c_double]
        lib.synth_batch_vertices.restype = ctypes.c_int64
        lib.synth_free.argtypes = [ctypes.c_void_p]
        lib.synth_free.restype = None
        _lib = lib
    return _lib


def _take_pairs(count: int, ptr) -> np.ndarray:
    lib = _load()
    if count < 0:
        raise MemoryError("synthetic generator failed (code %d)" % count)
    if count == 0:
        if ptr:
            lib.synth_free(ptr)
        return np.zeros((0, 2), dtype=np.int32)
    arr = np.ctypeslib.as_array(ptr, shape=(count * 2,)).copy().reshape(count, 2)
    lib.synth_free(ptr)
    return arr


@dataclass
class Graph:
    """Undirected simple graph as a symmetric CSR with sorted rows."""
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray      # int32[2m]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def neighbors(self, v: int) -> np.ndarray:
        return self.col[self.row_ptr[v]:self.row_ptr[v + 1]]

    def edges(self) -> np.ndarray:
        """Undirected edges (u < v), shape (m, 2)."""
        src = np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.row_ptr))
        keep = src < self.col
        return np.stack([src[keep], self.col[keep]], axis=1)


def from_pairs(n: int, pairs, name: str = "") -> Graph:
    """Canonical CSR from undirected pairs: symmetrised, self-loops and duplicates
    dropped, rows sorted ascending."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    if pairs.size and (pairs.min() < 0 or pairs.max() >= n):
        raise ValueError("vertex id out of range")
    u, v = pairs[:, 0], pairs[:, 1]
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.concatenate([u, v])
    b = np.concatenate([v, u])
    key = np.unique(a * n + b)
    src = (key // n).astype(np.int64)
    col = (key % n).astype(np.int32)
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("graph too large for int32 CSR")
    return Graph(n, row_ptr.astype(np.int32), col, name)


# ---------------------------------------------------------------- random graphs

def erdos_renyi(n: int, p: float, seed: int) -> Graph:
    lib = _load()
    ptr = ctypes.POINTER(ctypes.c_int32)()
    cnt = lib.synth_er(n, p, seed, ctypes.byref(ptr))
    return from_pairs(n, _take_pairs(cnt, ptr), "er(n=%d,p=%g,seed=%d)" % (n, p, seed))


def powerlaw_xmin(gamma: float, mean: float, xmax: float) -> float:
    """x_min of a power law w^(-gamma) truncated to [x_min, xmax] with the given mean
    (bisection on the closed-form mean)."""
    def mean_of(xmin):
        a = 1.0 - gamma
        norm = (xmax ** a - xmin ** a) / a
        b = 2.0 - gamma
        first = (xmax ** b - xmin ** b) / b if abs(b) > 1e-12 else math.log(xmax / xmin)
        return first / norm
    lo, hi = 1e-6, mean
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mean_of(mid) < mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def powerlaw_weights(n: int, gamma: float, mean: float, wmax: float, seed: int) -> np.ndarray:
    lib = _load()
    xmin = powerlaw_xmin(gamma, mean, wmax)
    w = np.empty(n, dtype=np.float64)
    lib.synth_powerlaw_weights(n, gamma, xmin, wmax, seed,
                               w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return w


def chung_lu_pairs(w: np.ndarray, seed: int) -> np.ndarray:
    lib = _load()
    w = np.ascontiguousarray(w, dtype=np.float64)
    ptr = ctypes.POINTER(ctypes.c_int32)()
    cnt = lib.synth_chung_lu(int(w.shape[0]), w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             seed, ctypes.byref(ptr))
    return _take_pairs(cnt, ptr)


def chung_lu(n: int, gamma: float, mean: float, wmax: float, seed: int) -> Graph:
    """Chung-Lu graph with i.i.d. power-law expected degrees (degree exponent gamma)."""
    w = powerlaw_weights(n, gamma, mean, wmax, seed)
    return from_pairs(n, chung_lu_pairs(w, seed),
                      "chung_lu(n=%d,gamma=%g,mean=%g,wmax=%g,seed=%d)" % (n, gamma, mean, wmax, seed))


def communities_pairs(n: int, nc: int, smin: int, smax: int, p: float, seed: int):
    lib = _load()
    sizes = np.zeros(max(nc, 1), dtype=np.int32)
    ptr = ctypes.POINTER(ctypes.c_int32)()
    cnt = lib.synth_communities(n, nc, smin, smax, p, seed,
                                sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                ctypes.byref(ptr))
    if cnt == -2:
        raise ValueError("communities do not fit in n")
    return _take_pairs(cnt, ptr), sizes[:nc]


def dense_core(n: int, mean: float, gamma: float, nc: int, smin: int, smax: int, p: float,
               seed: int, wmax: float = 0.0) -> Graph:
    """Chung-Lu background (w_max = sqrt(sum w) unless given, so no saturated
    core) plus `nc` planted communities with intra-density p."""
    wmax = wmax if wmax > 0 else math.sqrt(n * mean)
    w = powerlaw_weights(n, gamma, mean, wmax, seed)
    bg = chung_lu_pairs(w, seed)
    cm, _ = communities_pairs(n, nc, smin, smax, p, seed + 1)
    return from_pairs(n, np.concatenate([bg, cm]),
                      "dense_core(n=%d,mean=%g,nc=%d,size=[%d,%d],p=%g,seed=%d)"
                      % (n, mean, nc, smin, smax, p, seed))


def uniform(seed: int, i: int) -> float:
    return float(_load().synth_uniform(seed, i))


def permutation(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    _load().synth_permutation(n, seed, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return out


def relabel(g: Graph, seed: int) -> Graph:
    """Same graph under a random vertex relabelling."""
    perm = permutation(g.n, seed)
    e = g.edges().astype(np.int64)
    return from_pairs(g.n, perm[e], g.name + "|relabel%d" % seed)


# ------------------------------------------------------------ structured graphs

def empty(n: int) -> Graph:
    return from_pairs(n, np.zeros((0, 2), dtype=np.int64), "empty(%d)" % n)


def complete(n: int) -> Graph:
    iu = np.triu_indices(n, 1)
    return from_pairs(n, np.stack(iu, axis=1), "K%d" % n)


def complete_multipartite(parts) -> Graph:
    parts = list(parts)
    n = int(sum(parts))
    label = np.repeat(np.arange(len(parts)), parts)
    iu = np.triu_indices(n, 1)
    keep = label[iu[0]] != label[iu[1]]
    return from_pairs(n, np.stack([iu[0][keep], iu[1][keep]], axis=1),
                      "K(" + ",".join(map(str, parts)) + ")")


def cycle(n: int) -> Graph:
    a = np.arange(n)
    return from_pairs(n, np.stack([a, (a + 1) % n], axis=1), "C%d" % n)


def disjoint_union(g: Graph, h: Graph) -> Graph:
    e = np.concatenate([g.edges().astype(np.int64), h.edges().astype(np.int64) + g.n])
    return from_pairs(g.n + h.n, e, "(%s)+(%s)" % (g.name, h.name))


def join(g: Graph, h: Graph) -> Graph:
    """Disjoint union plus every edge between the two vertex sets."""
    a, b = np.meshgrid(np.arange(g.n), np.arange(h.n) + g.n, indexing="ij")
    cross = np.stack([a.ravel(), b.ravel()], axis=1)
    e = np.concatenate([g.edges().astype(np.int64), h.edges().astype(np.int64) + g.n, cross])
    return from_pairs(g.n + h.n, e, "(%s)v(%s)" % (g.name, h.name))


def random_bipartite(a: int, b: int, p: float, seed: int) -> Graph:
    g = erdos_renyi(a + b, p, seed)
    e = g.edges()
    side = e < a
    keep = side[:, 0] != side[:, 1]
    return from_pairs(a + b, e[keep], "bip(%d,%d,%g)" % (a, b, p))


# ---------------------------------------------------------------- batches

@dataclass
class Batch:
    """Independent graphs packed into one CSR: graph g owns vertices
    [voff[g], voff[g+1]) and its rows hold only its own vertices (global ids)."""
    voff: np.ndarray     # int32[ngraphs+1]
    row_ptr: np.ndarray  # int32[N+1]
    col: np.ndarray      # int32[nnz]

    @property
    def ngraphs(self) -> int:
        return int(self.voff.shape[0] - 1)

    @property
    def n(self) -> int:
        return int(self.voff[-1])

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def graph(self, g: int) -> Graph:
        a, b = int(self.voff[g]), int(self.voff[g + 1])
        rp = self.row_ptr[a:b + 1].astype(np.int64) - int(self.row_ptr[a])
        col = self.col[int(self.row_ptr[a]):int(self.row_ptr[b])] - a
        return Graph(b - a, rp.astype(np.int32), col.astype(np.int32), "batch[%d]" % g)


def batch(ngraphs: int, seed: int = 4, nmin: int = 50, nmax: int = 5000, dmin: float = 8.0,
          dmax: float = 64.0, gamma: float = 2.3) -> Batch:
    """Batched workload: `ngraphs` graphs with vertex counts log-uniform on
    [nmin, nmax], half Erdos-Renyi and half Chung-Lu (degree exponent gamma,
    weights capped at n - 1), mean degree uniform on [dmin, dmax] capped at
    n - 1, packed into one CSR."""
    lib = _load()
    V = int(lib.synth_batch_vertices(ngraphs, seed, nmin, nmax, dmin, dmax))
    voff = np.zeros(ngraphs + 1, dtype=np.int32)
    row_ptr = np.zeros(V + 1, dtype=np.int64)
    ptr = ctypes.POINTER(ctypes.c_int32)()
    nnz = lib.synth_batch(ngraphs, seed, nmin, nmax, dmin, dmax, gamma,
                          voff.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          row_ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(ptr))
    if nnz < 0:
        raise MemoryError("batch generation failed")
    if nnz > np.iinfo(np.int32).max:
        lib.synth_free(ptr)
        raise ValueError("batch too large for int32 CSR offsets")
    col = np.ctypeslib.as_array(ptr, shape=(max(nnz, 1),))[:nnz].copy()
    lib.synth_free(ptr)
    return Batch(voff, row_ptr.astype(np.int32), col)


# ------------------------------------------------------------- workload shapes

def config_small(seed: int = 1) -> Graph:
    """Erdos-Renyi G(2000, 0.01): the small plain-method workload."""
    return erdos_renyi(2000, 0.01, seed)


def config_densecore(seed: int = 3, n: int = 500_000, mean: float = 40.0, nc: int = 50, smin: int = 60,
                     smax: int = 80, p: float = 0.9, gamma: float = 2.1, wmax: float = 1000.0) -> Graph:
    """Dense-core workload: Chung-Lu background (n = 500k, mean degree 40, exponent
    2.1, expected degrees capped at 1000, so the background's own core stays small)
    plus 50 planted communities of U[smin, smax] vertices at intra-density 0.9.
    The default sizes are capped at 80 so that the single-threaded oracle counts
    every k within minutes (sizes of 100 and more hold 1e8 and more maximal cliques
    each)."""
    return dense_core(n, mean, gamma, nc, smin, smax, p, seed, wmax)


def config_powerlaw(seed: int = 2, n: int = 1_000_000, mean: float = 32.0,
                    wmax: float = 20000.0, gamma: float = 2.1) -> Graph:
    """Chung-Lu power-law workload: n = 1M, mean degree 32 (~16M edges), degree
    exponent 2.1, expected degrees capped at 20k."""
    return chung_lu(n, gamma, mean, wmax, seed)
