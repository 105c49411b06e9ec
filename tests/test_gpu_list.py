"""k-clique listing (kc_list) against independent enumerations.

Small graphs: the listed rows, as vertex sets, equal networkx's enumeration of
all cliques of size k (an enumerator that shares nothing with either side).
Larger graphs: every row is a k-clique of the input, no set repeats, and the
total equals the oracle's count.  Each row is in ascending orientation rank.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
networkx = pytest.importorskip("networkx")

SMALL = {
    "er_60": lambda: synth.erdos_renyi(60, 0.3, 5),
    "k12": lambda: synth.complete(12),
    "multipartite": lambda: synth.complete_multipartite((3, 3, 2, 4, 1)),
    "dense_core": lambda: synth.dense_core(400, 5.0, 2.1, 3, 12, 20, 0.9, 6),
    "cycle_and_isolated": lambda: synth.disjoint_union(synth.cycle(9), synth.empty(3)),
}


def nx_cliques(g, k):
    G = networkx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from(g.edges().tolist())
    return {tuple(sorted(c)) for c in networkx.enumerate_all_cliques(G) if len(c) == k}


def rank_of(kc, d):
    _, _, _, perm = kc.dag_to_host(d)
    rank = np.empty_like(perm)
    rank[perm] = np.arange(perm.size)
    return rank


def check_rows(g, rows, rank, k):
    """Every row is a k-clique of g, ascending in rank; returns the sorted rows."""
    rows = np.asarray(rows, dtype=np.int64).reshape(-1, k)
    if rows.size == 0:
        return rows
    assert rows.min() >= 0 and rows.max() < g.n
    if k > 1:
        assert np.all(np.diff(rank[rows], axis=1) > 0), "rows must ascend in orientation rank"
    e = g.edges().astype(np.int64)
    edge_keys = np.sort(e[:, 0] * g.n + e[:, 1])
    for a, b in itertools.combinations(range(k), 2):
        u, v = np.minimum(rows[:, a], rows[:, b]), np.maximum(rows[:, a], rows[:, b])
        assert np.isin(u * g.n + v, edge_keys, assume_unique=False).all(), "a listed row is not a clique"
    return np.sort(rows, axis=1)


@pytest.mark.parametrize("name", sorted(SMALL))
@pytest.mark.parametrize("scheme", [1, 2])
def test_listing_equals_enumeration(kc, name, scheme):
    g = SMALL[name]()
    for order in (kc.ORDER_DEGREE, kc.ORDER_DEGENERACY):
        d = kc.orient(kc.to_device(g), order)
        rank = rank_of(kc, d)
        for k in range(1, min(d.d_max + 2, 7) + 1):
            total, rows = kc.list_cliques(d, k, scheme=scheme)
            got = check_rows(g, rows.cpu().numpy(), rank, k)
            want = nx_cliques(g, k)
            assert total == len(want) == got.shape[0], (name, order, k)
            assert {tuple(r) for r in got.tolist()} == want, (name, order, k)


@pytest.mark.parametrize("scheme", [1, 2])
def test_listing_at_size(kc, scheme):
    # a power-law graph with a dense core: up to 5.7 million rows
    g = synth.chung_lu(4000, 2.1, 24.0, 600.0, 5)
    d = kc.orient(kc.to_device(g), kc.ORDER_DEGENERACY)
    od = oracle.orient(g, oracle.DEGENERACY)
    rank = rank_of(kc, d)
    for k in (3, 4, 5):
        want = oracle.count(od, k, False, oracle.VC)
        total, rows = kc.list_cliques(d, k, scheme=scheme)
        assert total == want == rows.shape[0], k
        got = check_rows(g, rows.cpu().numpy(), rank, k)
        assert np.unique(got, axis=0).shape[0] == want, "a clique is listed twice"


def test_listing_cap(kc):
    g = synth.chung_lu(4000, 2.1, 24.0, 600.0, 5)
    d = kc.orient(kc.to_device(g), kc.ORDER_DEGREE)
    rank = rank_of(kc, d)
    want = oracle.count(oracle.orient(g, oracle.DEGREE), 4, False, oracle.VC)
    for cap in (0, 1, 1000, want - 1, want, want + 5):
        st, total, rows = kc.list_cliques_status(d, 4, cap)
        assert st == kc.OK and total == want, cap
        assert rows.shape[0] == min(cap, want)
        got = check_rows(g, rows.cpu().numpy(), rank, 4)
        assert np.unique(got, axis=0).shape[0] == got.shape[0]


def test_listing_edge_cases(kc):
    import torch
    for g in (synth.empty(1), synth.empty(6), synth.complete(2), synth.cycle(5)):
        d = kc.orient(kc.to_device(g), kc.ORDER_DEGREE)
        for k in (1, 2, 3, 4):
            total, rows = kc.list_cliques(d, k)
            assert total == len(nx_cliques(g, k)) == rows.shape[0], (g.n, k)
    d = kc.orient(kc.to_device(synth.complete(10)), kc.ORDER_DEGREE)
    st, _, _ = kc.list_cliques_status(d, 0, 10)
    assert st == kc.EINVAL
    f = torch.ones(1, dtype=torch.int32, device="cuda")
    st, _, _ = kc.list_cliques_status(d, 4, 500, cancel=f.data_ptr())
    assert st == kc.ECANCELED
