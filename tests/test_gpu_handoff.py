"""The lane walk's subtree handoff between wavefronts, driven on purpose.

The ring queue only runs on width lists with fewer than two roots per
wavefront, once a walk has spent `handoff_after` rounds on its root.  The
dense-core workload with vertex roots puts its community vertices in the
4-word list and runs long enough at k >= 8 for the default thresholds; the
smaller heavy-core graph reaches the queue only with the thresholds lowered to
one round.  Every case checks the count against the oracle and that subtrees
were actually handed over (kc_profile.items_width).
"""
import pytest

import oracle
import synth
from conftest import load_counts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def densecore(kc):
    head, want, _ = load_counts("densecore_count_all.txt")
    g = synth.config_densecore()
    assert (g.n, g.m) == (head["n"], head["m"])
    return kc.orient(kc.to_device(g), kc.ORDER_DEGENERACY), want


@pytest.mark.parametrize("k", [8, 9, 10])
def test_densecore_vertex_roots_hand_over(kc, densecore, k):
    d, want = densecore
    p = kc.Profile()
    got = kc.count(d, k, pivot=False, scheme=kc.SCHEME_VC, profile=p)
    print("densecore VC k=%d items=%s" % (k, list(p.items_width)), flush=True)
    assert got == want[k]
    assert sum(p.items_width) > 0


def test_densecore_without_handoff(kc, densecore):
    d, want = densecore
    p = kc.Profile()
    assert kc.count(d, 10, pivot=False, scheme=kc.SCHEME_VC, profile=p, handoff=False) == want[10]
    assert sum(p.items_width) == 0


@pytest.mark.parametrize("k", range(4, 13))
def test_densecore_edge_roots(kc, densecore, k):
    d, want = densecore
    assert kc.count(d, k, pivot=False, scheme=kc.SCHEME_EC) == want[k]


@pytest.mark.parametrize("scheme", [1, 2])
def test_heavy_core_low_thresholds(kc, scheme):
    g = synth.dense_core(5000, 8.0, 2.1, 3, 150, 260, 0.45, 7)
    od = oracle.orient(g, oracle.DEGENERACY)
    d = kc.orient(kc.to_device(g), kc.ORDER_DEGENERACY)
    items = 0
    for k in (7, 8, 9):
        want = oracle.count(od, k, False, oracle.VC)
        for single in (False, True):
            p = kc.Profile()
            got = kc.count(d, k, pivot=False, scheme=scheme, profile=p, handoff_after=1, handoff_every=1,
                           single_stream=single)
            print("heavy_core scheme=%d k=%d single=%d items=%s" % (scheme, k, single, list(p.items_width)),
                  flush=True)
            assert got == want, (k, single)
            items += sum(p.items_width)
    assert items > 0
