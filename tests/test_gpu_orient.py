"""GPU orientation (kc_orient) against the oracle and the DAG invariants."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def gpu_dag(kc, g, order):
    return kc.orient(kc.to_device(g), order)


def check_dag(kc, g, d):
    rp, col, src, perm = kc.dag_to_host(d)
    assert d.n == g.n and d.m == g.m
    assert rp[0] == 0 and rp[-1] == g.m
    assert sorted(perm.tolist()) == list(range(g.n))
    if g.m:
        assert np.array_equal(src, np.repeat(np.arange(g.n), np.diff(rp)))
        assert np.all(col > src), "DAG edges must go from lower to higher new id"
        same_row = src[1:] == src[:-1]
        assert np.all(col[1:][same_row] > col[:-1][same_row]), "rows must be strictly increasing"
        back = np.sort(np.stack([perm[src], perm[col]], axis=1), axis=1)
        key = back[:, 0].astype(np.int64) * g.n + back[:, 1]
        e = g.edges()
        want = e[:, 0].astype(np.int64) * g.n + e[:, 1]
        assert np.array_equal(np.sort(key), np.sort(want))
    assert d.d_max == (int(np.diff(rp).max()) if g.n else 0)


GRAPHS = [
    lambda: synth.erdos_renyi(2000, 0.01, 1),
    lambda: synth.chung_lu(5000, 2.1, 16.0, 400.0, 2),
    lambda: synth.dense_core(6000, 10.0, 2.1, 5, 20, 40, 0.9, 3),
    lambda: synth.complete(50),
    lambda: synth.disjoint_union(synth.cycle(30), synth.empty(5)),
]


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_degree_order_matches_oracle(kc, gi):
    g = GRAPHS[gi]()
    d = gpu_dag(kc, g, kc.ORDER_DEGREE)
    check_dag(kc, g, d)
    od = oracle.orient(g, oracle.DEGREE)
    # degree order is (deg, id): the GPU relabelling equals the oracle's rank order
    _, _, _, perm = kc.dag_to_host(d)
    assert np.array_equal(perm, np.argsort(od.rank, kind="stable"))
    assert d.d_max == od.d_max


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_degeneracy_order(kc, gi):
    g = GRAPHS[gi]()
    d = gpu_dag(kc, g, kc.ORDER_DEGENERACY)
    check_dag(kc, g, d)
    od = oracle.orient(g, oracle.DEGENERACY)
    assert d.degeneracy == od.degeneracy          # the degeneracy itself is unique
    assert d.d_max <= d.degeneracy


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_approx_degeneracy_order_matches_oracle(kc, gi):
    # rounds of vertices at most 1.1 times the average degree: an integer rule,
    # so the GPU relabelling equals the oracle's (round, id) order bit for bit
    g = GRAPHS[gi]()
    d = gpu_dag(kc, g, kc.ORDER_APPROX_DEGENERACY)
    check_dag(kc, g, d)
    od = oracle.orient(g, oracle.APPROX_DEGENERACY)
    _, _, _, perm = kc.dag_to_host(d)
    assert np.array_equal(perm, np.argsort(od.rank, kind="stable"))
    assert d.d_max == od.d_max and d.degeneracy == -1
    for k in (3, 4, 5):
        want = oracle.count(od, k, False, oracle.VC)
        assert kc.count(d, k, pivot=False) == want, k
        assert kc.count(d, k, pivot=True) == want, k


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_colour_order_matches_oracle(kc, gi):
    # the greedy colouring by decreasing priority is unique (the priority is a
    # bijection of the id), so the Jones-Plassmann rounds must reproduce the
    # oracle's sequential colouring and its (colour, id) order bit for bit
    g = GRAPHS[gi]()
    d = gpu_dag(kc, g, kc.ORDER_COLOR)
    check_dag(kc, g, d)
    od = oracle.orient(g, oracle.COLOR)
    _, _, _, perm = kc.dag_to_host(d)
    assert np.array_equal(perm, np.argsort(od.rank, kind="stable"))
    assert d.d_max == od.d_max and d.degeneracy == -1
    for k in (3, 4, 5):
        want = oracle.count(od, k, False, oracle.VC)
        assert kc.count(d, k, pivot=False) == want, k
        assert kc.count(d, k, pivot=True) == want, k


def test_colour_order_complete_graph(kc):
    # K_n takes n rounds (one vertex per round) and n colours; d_max = n - 1 is
    # beyond the LDS limit, so the counts run through the wide roots
    import math
    n = 1500
    g = synth.complete(n)
    d = gpu_dag(kc, g, kc.ORDER_COLOR)
    _, _, _, perm = kc.dag_to_host(d)
    assert np.array_equal(perm, np.argsort(oracle.orient(g, oracle.COLOR).rank, kind="stable"))
    assert d.d_max == n - 1
    assert kc.count(d, 3, pivot=False) == math.comb(n, 3)
    assert kc.count(d, 6, pivot=True) == math.comb(n, 6)


def test_long_rows_sorted(kc):
    # DAG rows beyond 1024 entries are sorted by a block per row: bitonic in LDS
    # up to 8192 entries, rank placement beyond.  K_3000 in degree order has rows
    # of every length up to 2999; a star whose centre has the highest colouring
    # priority takes colour 0, so its row holds all 9000 leaves
    g = synth.complete(3000)
    d = gpu_dag(kc, g, kc.ORDER_DEGREE)
    check_dag(kc, g, d)
    assert d.d_max == 2999
    leaves = 9000
    centre = max(range(leaves + 1), key=lambda v: (oracle.splitmix64(v), v))
    star = synth.from_pairs(leaves + 1, [(centre, v) for v in range(leaves + 1) if v != centre])
    d = gpu_dag(kc, star, kc.ORDER_COLOR)
    check_dag(kc, star, d)
    assert d.d_max == leaves
    _, _, _, perm = kc.dag_to_host(d)
    assert perm[0] == centre
    assert np.array_equal(perm, np.argsort(oracle.orient(star, oracle.COLOR).rank, kind="stable"))


def test_colour_order_counts_at_size(kc):
    # the colouring DAG of the 1M-vertex power-law graph keeps hubs of up to 3779
    # out-neighbours, so its k = 4 count runs through the wide roots; the count
    # must equal the oracle's stored c_4 (counts do not depend on the order)
    from conftest import load_counts
    head, want, _ = load_counts("powerlaw_counts.txt")
    g = synth.config_powerlaw(wmax=5656.85424949238)
    assert (g.n, g.m) == (head["n"], head["m"])
    d = gpu_dag(kc, g, kc.ORDER_COLOR)
    assert d.d_max > kc.MAX_DMAX
    for scheme in (kc.SCHEME_VC, kc.SCHEME_EC):
        assert kc.count(d, 4, pivot=False, scheme=scheme) == want[4], scheme


def test_config_powerlaw_orientation(kc):
    g = synth.config_powerlaw(wmax=5657.0)
    for order in (kc.ORDER_DEGREE, kc.ORDER_DEGENERACY, kc.ORDER_APPROX_DEGENERACY, kc.ORDER_COLOR):
        d = gpu_dag(kc, g, order)
        check_dag(kc, g, d)
        od = oracle.orient(g, order)
        if order != kc.ORDER_DEGENERACY:
            _, _, _, perm = kc.dag_to_host(d)
            assert np.array_equal(perm, np.argsort(od.rank, kind="stable"))
            assert d.d_max == od.d_max
        else:
            assert d.degeneracy == od.degeneracy and d.d_max <= d.degeneracy


def test_empty_and_tiny(kc):
    for g in (synth.empty(1), synth.empty(7), synth.complete(2)):
        for order in (kc.ORDER_DEGREE, kc.ORDER_DEGENERACY, kc.ORDER_APPROX_DEGENERACY, kc.ORDER_COLOR):
            check_dag(kc, g, gpu_dag(kc, g, order))


def test_validation_rejects_malformed(kc):
    import torch
    g = synth.erdos_renyi(200, 0.05, 4)
    cases = []
    c = g.col.copy(); c[0], c[1] = c[1], c[0]; cases.append((g.row_ptr, c))          # unsorted row
    c = g.col.copy(); c[3] = g.n + 7; cases.append((g.row_ptr, c))                    # id out of range
    c = g.col.copy(); v = int(np.searchsorted(g.row_ptr, 5, side="right") - 1); c[5] = v; cases.append((g.row_ptr, c))  # self-loop
    rp = g.row_ptr.copy(); rp[10] = rp[11] + 3; cases.append((rp, g.col))             # non-monotone offsets
    e = g.edges()[1:]                                                                 # drop one direction of an edge
    und = synth.from_pairs(g.n, e)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    keep = ~((src == g.edges()[0][0]) & (g.col == g.edges()[0][1]))
    rp2 = np.concatenate([[0], np.cumsum(np.bincount(src[keep], minlength=g.n))]).astype(np.int32)
    cases.append((rp2, g.col[keep]))
    assert und.m == g.m - 1
    for rp_, col_ in cases:
        dev = kc.Csr(g.n, torch.as_tensor(np.ascontiguousarray(rp_, np.int32)).cuda(),
                     torch.as_tensor(np.ascontiguousarray(col_, np.int32)).cuda())
        with pytest.raises(kc.KcError) as e:
            kc.orient(dev, kc.ORDER_DEGREE, validate=True)
        assert e.value.code == kc.EINVAL


def test_degeneracy_order_repeatable(kc):
    """Repeated peels of the same graph into the same buffers give the identical
    permutation (the schedule is deterministic: keys are (round, id))."""
    import torch
    g = synth.config_powerlaw(wmax=5657.0)
    csr = kc.to_device(g)
    ws = torch.empty(kc.orient_workspace_bytes(g.n, g.nnz, kc.ORDER_DEGENERACY), dtype=torch.uint8, device="cuda")
    first = None
    for _ in range(6):
        d = kc.orient(csr, kc.ORDER_DEGENERACY, validate=True, ws=ws)
        assert d.d_max <= d.degeneracy
        perm = d.perm.cpu().numpy()
        if first is None:
            first = (perm, d.degeneracy, d.d_max)
        else:
            assert np.array_equal(perm, first[0]) and d.degeneracy == first[1] and d.d_max == first[2]
