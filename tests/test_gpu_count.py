"""GPU k-clique counts (kc_count) against the CPU oracle, element by element.

Counts are exact integers: the bar is equality.  Inputs are seeded synthetic
graphs chosen so that both root lists (light: |S| <= 64, one wavefront per root;
heavy: one workgroup per root) and several bitset words per row are exercised,
with ragged word counts.
"""
import math

import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def oracle_counts(g, ks):
    d = oracle.orient(g, oracle.DEGENERACY)
    return {k: oracle.count(d, k, False, oracle.VC) for k in ks}


SMALL = {
    "er_dense_40": lambda: synth.erdos_renyi(40, 0.6, 11),
    "er_2000": lambda: synth.erdos_renyi(2000, 0.01, 1),
    "chung_lu": lambda: synth.chung_lu(4000, 2.1, 24.0, 600.0, 5),
    "heavy_core": lambda: synth.dense_core(5000, 8.0, 2.1, 3, 150, 260, 0.45, 7),
    "dense_core": lambda: synth.dense_core(5000, 8.0, 2.1, 6, 30, 60, 0.85, 6),
    "k70": lambda: synth.complete(70),
    "multipartite": lambda: synth.complete_multipartite((3,) * 12 + (1, 2)),
}


@pytest.fixture(scope="module")
def cache():
    return {}


def get(cache, kc, name, order):
    key = (name, order)
    if key not in cache:
        g = SMALL[name]()
        cache[key] = (g, kc.orient(kc.to_device(g), order))
    return cache[key]


@pytest.mark.parametrize("name", sorted(SMALL))
@pytest.mark.parametrize("scheme", [1, 2])
def test_counts_match_oracle(kc, cache, name, scheme):
    for order in (kc.ORDER_DEGREE, kc.ORDER_DEGENERACY):
        g, d = get(cache, kc, name, order)
        kmax = min(d.d_max + 2, 8 if name != "k70" else 5)
        want = oracle_counts(g, range(1, kmax + 1))
        for k in range(1, kmax + 1):
            got = kc.count(d, k, pivot=False, scheme=scheme)
            assert got == want[k], (name, order, scheme, k)


@pytest.mark.parametrize("width", [0, 1, 2, 4, 8, 16, 32])
def test_widths_agree(kc, cache, width):
    # width 0/1: lane walks (pair tasks and helping at k >= 6 VC / 7 EC on wide roots);
    # 2..32: sub-wavefront groups
    g, d = get(cache, kc, "heavy_core", kc.ORDER_DEGENERACY)
    want = oracle_counts(g, (4, 6, 7))
    for scheme in (1, 2):
        for k in (4, 6, 7):
            assert kc.count(d, k, scheme=scheme, width=width) == want[k], (width, scheme, k)


@pytest.mark.parametrize("handoff,single_stream", [(True, False), (False, False), (True, True), (False, True)])
def test_scheduling_options_agree(kc, cache, handoff, single_stream):
    # deep counts on wide roots: subtree handoff between wavefronts, the widest
    # list on a side stream with a helper launch, or all on one stream
    g, d = get(cache, kc, "heavy_core", kc.ORDER_DEGENERACY)
    want = oracle_counts(g, (7, 8, 9))
    for scheme in (1, 2):
        for k in (7, 8, 9):
            got = kc.count(d, k, scheme=scheme, handoff=handoff, single_stream=single_stream)
            assert got == want[k], (handoff, single_stream, scheme, k)


def test_complete_graph_closed_form(kc):
    for n in (33, 64, 65, 100, 129, 200, 300, 520):
        g = synth.complete(n)
        d = kc.orient(kc.to_device(g), kc.ORDER_DEGREE)
        for k in ((3, 4, 5) if n <= 200 else (3, 4)):
            for scheme in (1, 2):
                assert kc.count(d, k, scheme=scheme) == math.comb(n, k), (n, k, scheme)


def test_edge_cases(kc):
    for g in (synth.empty(1), synth.empty(10), synth.cycle(12), synth.complete(2)):
        d = kc.orient(kc.to_device(g), kc.ORDER_DEGREE)
        for k in (1, 2, 3, 4):
            want = {1: g.n, 2: g.m}.get(k, 0)
            for scheme in (1, 2):
                assert kc.count(d, k, scheme=scheme) == want
    g = synth.complete(10)
    d = kc.orient(kc.to_device(g), kc.ORDER_DEGREE)
    assert kc.count(d, 11) == 0 and kc.count(d, 10) == 1
    st, _ = kc.count_status(d, 0)
    assert st == kc.EINVAL


def test_u64_overflow_is_reported(kc):
    g = synth.complete(12)
    d = kc.orient(kc.to_device(g), kc.ORDER_DEGREE)
    c4 = math.comb(12, 4)
    st, val = kc.count_status(d, 4, test_preload=2 ** 64 - c4)        # sum is exactly 2^64
    assert st == kc.EOVERFLOW
    st, val = kc.count_status(d, 4, test_preload=2 ** 64 - c4 - 1)    # sum is 2^64 - 1
    assert st == kc.OK and val == 2 ** 64 - 1


def test_repeatable(kc, cache):
    g, d = get(cache, kc, "dense_core", kc.ORDER_DEGENERACY)
    vals = {kc.count(d, 5, scheme=s, width=w) for s in (1, 2) for w in (2, 8) for _ in range(2)}
    assert len(vals) == 1


@pytest.mark.parametrize("name", sorted(n for n in SMALL if n not in ("k70", "chung_lu")))
@pytest.mark.parametrize("order", [0, 1])
def test_count_all_orientation_matches_oracle(kc, cache, name, order):
    # kc_count_all without pivoting: one orientation traversal per size (K_70
    # and the Chung-Lu graph, with 1e21 and 8e11 cliques, are left to pivoting)
    g, d = get(cache, kc, name, order)
    want, om = oracle.count_all(oracle.orient(g, oracle.DEGENERACY), True, oracle.VC)
    got, gom = kc.count_all(d, pivot=False, cap=d.d_max + 2)
    assert gom == om, name
    assert got[:om + 1] == want[:om + 1], name
    assert all(c == 0 for c in got[om + 1:])
    # a cap below omega keeps the exact omega and the counts up to the cap
    if om > 3:
        got, gom = kc.count_all(d, pivot=False, cap=3)
        assert gom == om and got == want[:4]


@pytest.mark.parametrize("name", sorted(SMALL))
@pytest.mark.parametrize("scheme", [1, 2])
def test_list_intersection_ablation_matches_oracle(kc, cache, name, scheme):
    # KC_OPT_NO_BITSETS: sorted lists and binary-search intersections instead of
    # bitset rows (the paper's non-binary-encoded variant)
    for order in (kc.ORDER_DEGREE, kc.ORDER_DEGENERACY):
        g, d = get(cache, kc, name, order)
        kmax = min(d.d_max + 2, 8 if name != "k70" else 5)
        want = oracle_counts(g, range(3, kmax + 1))
        for k in range(3, kmax + 1):
            assert kc.count(d, k, pivot=False, scheme=scheme, bitsets=False) == want[k], (name, order, scheme, k)
