"""GPU pivoting counts (kc_count with pivot, kc_count_all) against the CPU oracle.

Counts are exact: equality is the bar.  The 64/128-bit boundary cases use the
closed form C(n, k) on complete graphs, where the pivot tree is one path.
"""
import math

import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GRAPHS = {
    "er_dense_40": lambda: synth.erdos_renyi(40, 0.6, 11),
    "er_2000": lambda: synth.erdos_renyi(2000, 0.01, 1),
    "chung_lu": lambda: synth.chung_lu(4000, 2.1, 24.0, 600.0, 5),
    "heavy_core": lambda: synth.dense_core(5000, 8.0, 2.1, 3, 150, 260, 0.45, 7),
    "communities": lambda: synth.dense_core(20000, 10.0, 2.1, 6, 40, 75, 0.9, 8),
    "moon_moser": lambda: synth.complete_multipartite((3,) * 14),
}


@pytest.fixture(scope="module")
def cache():
    return {}


def get(cache, kc, name, order):
    key = (name, order)
    if key not in cache:
        g = GRAPHS[name]()
        od = oracle.orient(g, oracle.DEGENERACY)
        want, om = oracle.count_all(od, True, oracle.VC)
        cache[key] = (g, kc.orient(kc.to_device(g), order), want, om)
    return cache[key]


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("scheme", [1, 2])
def test_pivot_count_matches_oracle(kc, cache, name, scheme):
    for order in (kc.ORDER_DEGREE, kc.ORDER_DEGENERACY):
        g, d, want, om = get(cache, kc, name, order)
        for k in range(1, om + 2):
            assert kc.count(d, k, pivot=True, scheme=scheme) == (want[k] if k < len(want) else 0), (name, order, k)


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("scheme", [1, 2])
def test_count_all_matches_oracle(kc, cache, name, scheme):
    for order in (kc.ORDER_DEGREE, kc.ORDER_DEGENERACY):
        g, d, want, om = get(cache, kc, name, order)
        got, gom = kc.count_all(d, pivot=True, scheme=scheme)
        assert gom == om
        assert got[:len(want)] == want[:len(got)], (name, order)
        assert all(x == 0 for x in got[len(want):])


def test_pivot_agrees_with_orientation(kc, cache):
    g, d, want, om = get(cache, kc, "heavy_core", kc.ORDER_DEGENERACY)
    for k in (3, 4, 5, 6):
        assert kc.count(d, k, pivot=True) == kc.count(d, k, pivot=False)


def test_complete_graphs_and_128_bit_boundary(kc):
    d = kc.orient(kc.to_device(synth.complete(68)), kc.ORDER_DEGREE)
    assert kc.count(d, 34, pivot=True) == math.comb(68, 34) > 2 ** 64
    d = kc.orient(kc.to_device(synth.complete(131)), kc.ORDER_DEGENERACY)
    got, om = kc.count_all(d, pivot=True)
    assert om == 131 and got[:132] == [math.comb(131, j) for j in range(132)]
    for k in (2, 3, 65, 66, 130, 131, 132):
        assert kc.count(d, k, pivot=True) == math.comb(131, k)
    d = kc.orient(kc.to_device(synth.complete(132)), kc.ORDER_DEGREE)
    with pytest.raises(kc.KcError) as e:
        kc.count_all(d, pivot=True)
    assert e.value.code == kc.EOVERFLOW
    assert kc.count(d, 5, pivot=True) == math.comb(132, 5)
    st, _ = kc.count_status(d, 66, pivot=True)
    assert st == kc.EOVERFLOW


def test_pivot_edge_cases(kc):
    for g in (synth.empty(1), synth.empty(9), synth.cycle(15), synth.complete(2), synth.complete(3)):
        d = kc.orient(kc.to_device(g), kc.ORDER_DEGENERACY)
        bc = oracle.brute_counts(g)
        got, om = kc.count_all(d, pivot=True, cap=6)
        assert got == (bc + [0] * 7)[:7]
        for k in (1, 2, 3, 4):
            assert kc.count(d, k, pivot=True) == (bc[k] if k < len(bc) else 0)


def _densecore_fixture():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "densecore_count_all.txt")
    head, counts = {}, {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "c":
                counts[int(parts[1])] = int(parts[2])
            else:
                head[parts[0]] = int(parts[1])
    return head, counts


def test_config_densecore_count_all(kc):
    # the dense-core workload at full size (n = 500k, ~10M edges, 50 planted
    # communities): every c_k against the oracle's counts stored by
    # tests/golden/make_densecore_counts.py, in both root schemes
    head, want = _densecore_fixture()
    g = synth.config_densecore()
    assert (g.n, g.m) == (head["n"], head["m"])
    d = kc.orient(kc.to_device(g), kc.ORDER_DEGENERACY)
    for scheme in (kc.SCHEME_VC, kc.SCHEME_EC):
        got, omega = kc.count_all(d, pivot=True, scheme=scheme)
        assert omega == head["omega"], scheme
        assert got[:omega + 1] == [want[k] for k in range(omega + 1)], scheme
        assert all(c == 0 for c in got[omega + 1:])
