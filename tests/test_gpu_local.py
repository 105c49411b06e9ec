"""Per-vertex k-clique counts (kc_count_local) against the oracle's local counts,
element by element, with and without pivoting, vertex and edge roots, both
orientations; and the sum rule sum_v local_v = k * c_k."""
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GRAPHS = {
    "er_dense_40": lambda: synth.erdos_renyi(40, 0.6, 11),
    "er_2000": lambda: synth.erdos_renyi(2000, 0.01, 1),
    "chung_lu": lambda: synth.chung_lu(4000, 2.1, 24.0, 600.0, 5),
    "heavy_core": lambda: synth.dense_core(5000, 8.0, 2.1, 3, 150, 260, 0.45, 7),
    "dense_core": lambda: synth.dense_core(5000, 8.0, 2.1, 6, 30, 60, 0.85, 6),
    "multipartite": lambda: synth.complete_multipartite((3,) * 12 + (1, 2)),
    "k40": lambda: synth.complete(40),
}


@pytest.fixture(scope="module")
def cache():
    return {}


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("order", [0, 1])
def test_local_counts_match_oracle(kc, cache, name, order):
    if name not in cache:
        g = GRAPHS[name]()
        cache[name] = (g, oracle.orient(g, oracle.DEGENERACY))
    g, od = cache[name]
    d = kc.orient(kc.to_device(g), order)
    kmax = min(d.d_max + 2, 7)
    for k in range(1, kmax + 1):
        want = oracle.count_local(od, k)
        total = oracle.count(od, k, False, oracle.VC)
        assert sum(want) == k * total
        for pivot in (False, True):
            for scheme in (1, 2):
                got = [int(x) & ((1 << 64) - 1) for x in kc.count_local(d, k, pivot, scheme).cpu().tolist()]
                assert got == want, (name, order, k, pivot, scheme)


def test_local_counts_edge_cases(kc):
    for g in (synth.empty(5), synth.complete(3), synth.cycle(9)):
        d = kc.orient(kc.to_device(g), kc.ORDER_DEGENERACY)
        od = oracle.orient(g, oracle.DEGENERACY)
        for k in range(1, 6):
            for pivot in (False, True):
                got = [int(x) for x in kc.count_local(d, k, pivot).cpu().tolist()]
                assert got == oracle.count_local(od, k), (g.name, k, pivot)
