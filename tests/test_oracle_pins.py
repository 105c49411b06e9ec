"""Pins of the CPU oracle against what the paper and mathematics fix.

Nothing here compares the oracle with itself: every expected value comes from
brute-force enumeration (two independent enumerators), a closed form, a library
routine (networkx), linear algebra, or the paper's own worked instance.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
import synth

networkx = pytest.importorskip("networkx")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MODES = [(p, s) for p in (False, True) for s in (oracle.VC, oracle.EC)]
ORDERS = (oracle.DEGREE, oracle.DEGENERACY)


def all_counts(g, order, pivot, scheme, kmax):
    d = oracle.orient(g, order)
    return [oracle.count(d, k, pivot, scheme) for k in range(1, kmax + 1)]


def py_brute(g):
    """Pure-Python enumeration over vertex subsets (tiny graphs only)."""
    adj = [set(g.neighbors(v).tolist()) for v in range(g.n)]
    out = [1] + [0] * g.n
    for k in range(1, g.n + 1):
        for sub in itertools.combinations(range(g.n), k):
            if all(b in adj[a] for a, b in itertools.combinations(sub, 2)):
                out[k] += 1
    return out


def to_nx(g):
    G = networkx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from(g.edges().tolist())
    return G


def elem_sym(xs, k):
    e = [1] + [0] * len(xs)
    for x in xs:
        for j in range(len(xs), 0, -1):
            e[j] += e[j - 1] * x
    return e[k] if k <= len(xs) else 0


# ------------------------------------------------------------ brute force

def test_brute_enumerators_agree():
    """The two independent brute-force enumerators agree (C bitmask DFS vs Python subsets)."""
    for seed in range(12):
        g = synth.erdos_renyi(12, 0.15 + 0.06 * seed, seed)
        assert oracle.brute_counts(g) == py_brute(g)


@pytest.mark.parametrize("seed", range(40))
def test_counts_match_brute_force_random(seed):
    n = 10 + (seed * 7) % 31              # 10..40 vertices
    p = 0.1 + 0.8 * ((seed * 13) % 9) / 8.0
    g = synth.erdos_renyi(n, p, 1000 + seed)
    want = oracle.brute_counts(g)
    kmax = max(k for k in range(len(want)) if want[k]) + 1
    for order in ORDERS:
        for pivot, scheme in MODES:
            got = all_counts(g, order, pivot, scheme, kmax)
            assert got == want[1:kmax + 1], (order, pivot, scheme)


@pytest.mark.parametrize("seed", range(6))
def test_count_all_matches_brute_force(seed):
    g = synth.erdos_renyi(36, 0.5 + 0.08 * seed, 50 + seed)
    want = oracle.brute_counts(g)
    for order in ORDERS:
        d = oracle.orient(g, order)
        for pivot, scheme in MODES:
            got, om = oracle.count_all(d, pivot, scheme, cap=g.n)
            assert got == want, (order, pivot, scheme)
            assert om == max(k for k in range(len(want)) if want[k])


def test_counts_match_networkx_cliques():
    for seed in range(4):
        g = synth.erdos_renyi(60, 0.3 + 0.1 * seed, 77 + seed)
        hist = {}
        for c in networkx.enumerate_all_cliques(to_nx(g)):
            hist[len(c)] = hist.get(len(c), 0) + 1
        d = oracle.orient(g, oracle.DEGENERACY)
        for k in range(1, max(hist) + 2):
            for pivot, scheme in MODES:
                assert oracle.count(d, k, pivot, scheme) == hist.get(k, 0)


def test_triangles_trace_formula():
    """c_3 = trace(A^3) / 6."""
    for seed in range(5):
        g = synth.erdos_renyi(120, 0.12, 300 + seed)
        A = np.zeros((g.n, g.n), dtype=np.int64)
        e = g.edges()
        A[e[:, 0], e[:, 1]] = 1
        A[e[:, 1], e[:, 0]] = 1
        want = int(np.trace(A @ A @ A)) // 6
        d = oracle.orient(g, oracle.DEGREE)
        for pivot, scheme in MODES:
            assert oracle.count(d, 3, pivot, scheme) == want


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 9, 17, 30])
def test_complete_graph(n):
    g = synth.complete(n)
    for order in ORDERS:
        d = oracle.orient(g, order)
        assert d.d_max == n - 1
        for pivot, scheme in MODES:
            for k in range(1, n + 2):
                if not pivot and n > 20 and 6 < k:
                    continue   # the orientation tree of K_30 beyond k = 6 is large; pivot covers it
                assert oracle.count(d, k, pivot, scheme) == math.comb(n, k), (order, pivot, scheme, k)


def test_k3_reading_of_fig3():
    """K_3 under the l-reading of Fig. 3: 3 vertices, 3 edges, 1 triangle."""
    d = oracle.orient(synth.complete(3), oracle.DEGREE)
    for scheme in (oracle.VC, oracle.EC):
        assert [oracle.count(d, k, True, scheme) for k in (1, 2, 3, 4)] == [3, 3, 1, 0]


@pytest.mark.parametrize("parts", [(1, 1), (2, 3), (3, 3, 3), (1, 2, 3, 4), (5, 1, 5, 2, 2), (2,) * 8, (3,) * 7])
def test_complete_multipartite(parts):
    """c_k of a complete multipartite graph is the elementary symmetric polynomial e_k(parts)."""
    g = synth.complete_multipartite(parts)
    for order in ORDERS:
        d = oracle.orient(g, order)
        for pivot, scheme in MODES:
            for k in range(1, len(parts) + 2):
                assert oracle.count(d, k, pivot, scheme) == elem_sym(parts, k)


def test_cocktail_party_and_moon_moser():
    # cocktail party graph K_{2,...,2} (r parts): C(r, k) 2^k; Moon-Moser K_{3,...,3}: C(r, k) 3^k
    for size, r in ((2, 9), (3, 6)):
        d = oracle.orient(synth.complete_multipartite((size,) * r), oracle.DEGENERACY)
        c, om = oracle.count_all(d, True, oracle.VC)
        assert om == r
        assert c[:r + 1] == [math.comb(r, k) * size ** k for k in range(r + 1)]


def test_join_convolution():
    """c_k(G v H) = sum_i c_i(G) c_{k-i}(H) with c_0 = 1."""
    for seed in range(4):
        G = synth.erdos_renyi(14, 0.45, 900 + seed)
        H = synth.erdos_renyi(12, 0.55, 950 + seed)
        cg, ch = oracle.brute_counts(G), oracle.brute_counts(H)
        J = synth.join(G, H)
        want = [sum(cg[i] * ch[k - i] for i in range(k + 1) if i < len(cg) and k - i < len(ch))
                for k in range(J.n + 1)]
        for order in ORDERS:
            d = oracle.orient(J, order)
            for pivot, scheme in MODES:
                got, _ = oracle.count_all(d, pivot, scheme, cap=J.n)
                assert got == want


def test_disjoint_union_sums():
    G = synth.erdos_renyi(30, 0.4, 5)
    H = synth.complete(7)
    U = synth.disjoint_union(G, H)
    cg, ch = oracle.brute_counts(G), [math.comb(7, k) for k in range(8)]
    d = oracle.orient(U, oracle.DEGENERACY)
    for k in range(1, 9):
        want = (cg[k] if k < len(cg) else 0) + (ch[k] if k < len(ch) else 0)
        for pivot, scheme in MODES:
            assert oracle.count(d, k, pivot, scheme) == want


def test_triangle_free_graphs():
    for g in (synth.cycle(50), synth.random_bipartite(40, 30, 0.3, 4), synth.empty(20)):
        d = oracle.orient(g, oracle.DEGREE)
        for pivot, scheme in MODES:
            assert oracle.count(d, 1, pivot, scheme) == g.n
            assert oracle.count(d, 2, pivot, scheme) == g.m
            for k in (3, 4, 5):
                assert oracle.count(d, k, pivot, scheme) == 0


def test_paper_five_clique_fixture():
    """Sec. 2.3: the 5-clique {A,B,C,D,J} holds C(5,4) = 5 four-cliques."""
    lines = [l.split() for l in open(os.path.join(GOLDEN, "paper_five_clique.txt")) if l.strip() and l[0] != "#"]
    names = lines[0][1:]
    idx = {v: i for i, v in enumerate(names)}
    edges = [(idx[a], idx[b]) for a, b in (l for l in lines[1:] if l[0] != "count")]
    g = synth.from_pairs(len(names), edges)
    for l in lines:
        if l[0] == "count":
            k, val = int(l[1]), int(l[2])
            for order in ORDERS:
                d = oracle.orient(g, order)
                for pivot, scheme in MODES:
                    assert oracle.count(d, k, pivot, scheme) == val


# ------------------------------------------------------------- invariants

def test_local_counts_sum_and_agree():
    for seed in range(5):
        g = synth.erdos_renyi(45, 0.45, 60 + seed)
        tri = networkx.triangles(to_nx(g))
        deg = g.degrees()
        for k in range(1, 8):
            ref = None
            total = None
            for order in ORDERS:
                d = oracle.orient(g, order)
                for pivot, scheme in MODES:
                    loc = oracle.count_local(d, k, pivot, scheme)
                    if ref is None:
                        ref = loc
                        total = oracle.count(d, k, pivot, scheme)
                    assert loc == ref, (k, order, pivot, scheme)
                    assert sum(loc) == k * total
            if k == 2:
                assert ref == deg.tolist()
            if k == 3:
                assert ref == [tri[v] for v in range(g.n)]


def test_local_counts_brute():
    g = synth.erdos_renyi(18, 0.6, 7)
    adj = [set(g.neighbors(v).tolist()) for v in range(g.n)]
    for k in (3, 4, 5):
        want = [0] * g.n
        for sub in itertools.combinations(range(g.n), k):
            if all(b in adj[a] for a, b in itertools.combinations(sub, 2)):
                for v in sub:
                    want[v] += 1
        d = oracle.orient(g, oracle.DEGENERACY)
        for pivot, scheme in MODES:
            assert oracle.count_local(d, k, pivot, scheme) == want


def dag_checks(g, d):
    rp, col, rank = d.row_ptr, d.col, d.rank
    m = g.m
    assert rp[-1] == m
    src = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(rank[src] < rank[col]), "rank must increase along every DAG edge"
    und = {(min(a, b), max(a, b)) for a, b in zip(src.tolist(), col.tolist())}
    assert len(und) == m and und == {tuple(e) for e in g.edges().tolist()}
    assert sorted(rank.tolist()) == list(range(g.n))


def test_orientation_invariants():
    for seed in range(4):
        for g in (synth.erdos_renyi(300, 0.05, seed), synth.chung_lu(3000, 2.1, 12.0, 300.0, seed)):
            dd = oracle.orient(g, oracle.DEGREE)
            dag_checks(g, dd)
            assert dd.d_max <= math.isqrt(2 * g.m) + 1
            dg = oracle.orient(g, oracle.DEGENERACY)
            dag_checks(g, dg)
            core = max(networkx.core_number(to_nx(g)).values()) if g.m else 0
            assert dg.degeneracy == core
            assert dg.d_max == core


def test_degree_order_is_lexicographic():
    g = synth.chung_lu(500, 2.3, 8.0, 60.0, 9)
    d = oracle.orient(g, oracle.DEGREE)
    deg = g.degrees()
    order = sorted(range(g.n), key=lambda v: (deg[v], v))
    assert [int(d.rank[v]) for v in order] == list(range(g.n))


def test_relabel_invariance():
    g = synth.chung_lu(800, 2.1, 14.0, 120.0, 3)
    h = synth.relabel(g, 17)
    for order in ORDERS:
        a = oracle.orient(g, order)
        b = oracle.orient(h, order)
        for k in (3, 4, 5):
            assert oracle.count(a, k, False, oracle.VC) == oracle.count(b, k, True, oracle.EC)


# ------------------------------------------- approximate degeneracy order

def test_approx_degeneracy_hand_cases():
    # regular graphs: every vertex leaves in round 0, so the order is the id order
    for g in (synth.cycle(9), synth.complete(7), synth.complete_multipartite((2,) * 5)):
        d = oracle.orient(g, oracle.APPROX_DEGENERACY)
        assert [int(x) for x in d.rank] == list(range(g.n))
        assert d.degeneracy == -1
    # star K_{1,5}, centre 0: round 0 (L = 6, D = 10) removes the leaves
    # (10 * 1 * 6 <= 110) but not the centre (10 * 5 * 6 = 300 > 110)
    star = synth.from_pairs(6, [(0, i) for i in range(1, 6)])
    d = oracle.orient(star, oracle.APPROX_DEGENERACY)
    assert [int(x) for x in d.rank] == [5, 0, 1, 2, 3, 4]
    # broom: K_5 on 0..4 and 20 pendant vertices 5..24 on vertex 0.  Round 0:
    # L = 25, D = 60, 10 deg 25 <= 660 keeps degree <= 2: the pendants.  Round 1:
    # K_5 alone (L = 5, D = 20, 10 * 4 * 5 <= 220) leaves at once, in id order.
    pairs = [(a, b) for a in range(5) for b in range(a + 1, 5)] + [(0, i) for i in range(5, 25)]
    d = oracle.orient(synth.from_pairs(25, pairs), oracle.APPROX_DEGENERACY)
    assert [int(x) for x in d.rank] == [20, 21, 22, 23, 24] + list(range(20))


def test_approx_degeneracy_bound_and_counts():
    # a vertex leaves with at most 1.1 times the average degree of what remains,
    # and every sub-graph's average degree is at most twice the degeneracy, so
    # degeneracy <= d_max <= 2.2 * degeneracy; counts do not depend on the order
    for seed in range(3):
        for g in (synth.erdos_renyi(300, 0.05, seed), synth.chung_lu(3000, 2.1, 12.0, 300.0, seed),
                  synth.dense_core(3000, 6.0, 2.1, 3, 30, 50, 0.8, seed)):
            da = oracle.orient(g, oracle.APPROX_DEGENERACY)
            dag_checks(g, da)
            core = oracle.orient(g, oracle.DEGENERACY).degeneracy
            assert core <= da.d_max and 5 * da.d_max <= 11 * core
            dd = oracle.orient(g, oracle.DEGREE)
            for k in (3, 4, 5):
                assert oracle.count(da, k, False, oracle.VC) == oracle.count(dd, k, True, oracle.EC)


# --------------------------------------------------------- colouring order

def test_splitmix64_published_vectors():
    # SplitMix64 seeded with 0 first returns 0xE220A8397B1DCDAF; seeded with
    # 1234567 it returns the five values below (outputs of its published
    # reference implementation).  The oracle's function is the output for the
    # state before the increment, so the i-th output is f(seed + (i - 1) gamma).
    gamma = 0x9E3779B97F4A7C15
    assert oracle.splitmix64(0) == 0xE220A8397B1DCDAF
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    got = [oracle.splitmix64((1234567 + i * gamma) % 2 ** 64) for i in range(5)]
    assert got == want


def _priority_order(n):
    return sorted(range(n), key=lambda v: (oracle.splitmix64(v), v), reverse=True)


def test_colouring_closed_forms():
    # K_n: every vertex sees all earlier ones, so its colour is its place in the
    # decreasing-priority order, and the orientation follows that order
    n = 40
    c = oracle.colour(synth.complete(n))
    order = _priority_order(n)
    assert [int(c[v]) for v in order] == list(range(n))
    d = oracle.orient(synth.complete(n), oracle.COLOR)
    assert [int(d.rank[v]) for v in order] == list(range(n))
    # complete multipartite: greedy gives every part one colour (vertices of a
    # part have equal neighbourhoods), so exactly as many colours as parts, and
    # parts are coloured in the order their first vertex appears
    parts = (3, 1, 4, 1, 5, 9, 2, 6)
    g = synth.complete_multipartite(parts)
    c = oracle.colour(g)
    part_of = np.repeat(np.arange(len(parts)), parts)
    assert len(set(c.tolist())) == len(parts)
    for p_ in range(len(parts)):
        assert len(set(c[part_of == p_].tolist())) == 1
    first_seen = []
    for v in _priority_order(g.n):
        if part_of[v] not in first_seen:
            first_seen.append(part_of[v])
    assert [int(c[np.flatnonzero(part_of == p_)[0]]) for p_ in first_seen] == list(range(len(parts)))
    # independent set: one colour, order = id order
    d = oracle.orient(synth.empty(9), oracle.COLOR)
    assert [int(x) for x in d.rank] == list(range(9))


def test_colouring_is_lexicographically_least():
    # Visiting vertices in priority order, first fit yields the lexicographically
    # least proper colouring of that sequence; brute force over all colourings
    for seed in range(6):
        g = synth.erdos_renyi(6, 0.5, seed)
        order = _priority_order(g.n)
        edges = g.edges().tolist()
        best = None
        for cols in itertools.product(range(g.n), repeat=g.n):
            if all(cols[a] != cols[b] for a, b in edges):
                seq = tuple(cols[v] for v in order)
                if best is None or seq < best:
                    best = seq
        c = oracle.colour(g)
        assert tuple(int(c[v]) for v in order) == best, seed


def test_colouring_order_invariants_and_counts():
    for seed in range(3):
        for g in (synth.erdos_renyi(300, 0.05, seed), synth.chung_lu(3000, 2.1, 12.0, 300.0, seed)):
            c = oracle.colour(g)
            e = g.edges()
            assert np.all(c[e[:, 0]] != c[e[:, 1]]), "proper colouring"
            deg = np.diff(g.row_ptr)
            assert np.all(c <= deg), "first fit uses at most deg + 1 colours at a vertex"
            d = oracle.orient(g, oracle.COLOR)
            dag_checks(g, d)
            assert d.degeneracy == -1
            # (colour, id) order
            assert np.array_equal(np.argsort(d.rank), np.lexsort((np.arange(g.n), c)))
            dd = oracle.orient(g, oracle.DEGREE)
            for k in (3, 4, 5):
                assert oracle.count(d, k, False, oracle.VC) == oracle.count(dd, k, True, oracle.EC)


# ------------------------------------------------------------- arithmetic

def test_u128_boundaries():
    # K_68: C(68, 34) > 2^64 but fits 128 bits; K_131 fits, K_132 overflows 128 bits
    d = oracle.orient(synth.complete(68), oracle.DEGREE)
    assert oracle.count(d, 34, True, oracle.VC) == math.comb(68, 34) > 2 ** 64
    d = oracle.orient(synth.complete(131), oracle.DEGREE)
    c, om = oracle.count_all(d, True, oracle.VC)
    assert om == 131 and c[:132] == [math.comb(131, j) for j in range(132)]
    assert max(c) < 2 ** 128
    d = oracle.orient(synth.complete(132), oracle.DEGREE)
    with pytest.raises(oracle.OracleError) as e:
        oracle.count_all(d, True, oracle.VC)
    assert e.value.code == oracle.EOVERFLOW
    assert oracle.count(d, 3, True, oracle.VC) == math.comb(132, 3)


def test_root_subsets_partition_the_count():
    g = synth.chung_lu(2000, 2.1, 10.0, 150.0, 11)
    d = oracle.orient(g, oracle.DEGENERACY)
    for scheme, nroots in ((oracle.VC, g.n), (oracle.EC, d.m)):
        total = oracle.count(d, 4, False, scheme)
        perm = np.random.default_rng(0).permutation(nroots)
        parts = np.array_split(perm, 5)
        assert sum(oracle.count(d, 4, False, scheme, roots=p) for p in parts) == total


def test_validate_rejects_malformed():
    g = synth.erdos_renyi(30, 0.3, 1)
    assert oracle.validate(g)
    bad = synth.Graph(g.n, g.row_ptr.copy(), g.col.copy())
    bad.col[0], bad.col[1] = bad.col[1], bad.col[0]     # unsorted row
    assert not oracle.validate(bad)
    asym = synth.Graph(3, np.array([0, 1, 1, 1], np.int32), np.array([1], np.int32))
    assert not oracle.validate(asym)
