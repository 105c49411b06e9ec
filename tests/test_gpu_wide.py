"""Wide roots: roots whose first vertex has more than 1024 out-neighbours, so that
their candidate sets are encoded in a global-memory slab per wavefront instead of
LDS (both the orientation walk of Fig. 2 and the pivot walk of Fig. 3).

Expected values hold for the whole graph and do not come from the GPU:
  * K_n: c_k = C(n, k);
  * the cocktail-party graph on m pairs: c_k = C(m, k) 2^k;
  * G joined with an independent set of b vertices: a clique holds at most one
    vertex of the independent set, so c_k = c_k(G) + b c_{k-1}(G), with c(G) from
    the oracle on G alone (the oracle on the whole join takes minutes).
Counts are exact integers: the bar is equality.
"""
import math

import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

JOIN_B = 1200


@pytest.fixture(scope="module")
def join(kc):
    ga = synth.erdos_renyi(1100, 0.1, 21)
    g = synth.join(ga, synth.empty(JOIN_B))
    ca, om = oracle.count_all(oracle.orient(ga, oracle.DEGENERACY), True, oracle.VC)
    want = [1, g.n, len(g.col) // 2] + [ca[k] + JOIN_B * ca[k - 1] for k in range(3, om + 3)]
    while want[-1] == 0:
        want.pop()
    dev = kc.to_device(g)
    dags = {order: kc.orient(dev, order) for order in (kc.ORDER_DEGREE, kc.ORDER_DEGENERACY)}
    return want, dags


@pytest.fixture(scope="module")
def complete(kc):
    out = {}
    for n in (1100, 2100):
        out[n] = kc.orient(kc.to_device(synth.complete(n)), kc.ORDER_DEGREE)
    return out


def test_join_has_wide_roots(kc, join):
    want, dags = join
    assert len(want) - 1 == 7                     # omega of the join
    for d in dags.values():
        assert kc.MAX_DMAX < d.d_max <= kc.MAX_DMAX_WIDE


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("scheme", [1, 2])
def test_join_counts(kc, join, order, scheme):
    want, dags = join
    d = dags[order]
    for k in range(3, 7):
        assert kc.count(d, k, pivot=False, scheme=scheme) == want[k], ("orientation", k)
    for k in range(3, 9):
        exp = want[k] if k < len(want) else 0
        assert kc.count(d, k, pivot=True, scheme=scheme) == exp, ("pivot", k)
    got, om = kc.count_all(d, pivot=True, scheme=scheme)
    assert om == len(want) - 1
    assert got[:om + 1] == want


def test_join_count_all_orientation(kc, join):
    want, dags = join
    got, om = kc.count_all(dags[kc.ORDER_DEGREE], pivot=False, scheme=kc.SCHEME_VC)
    assert om == len(want) - 1
    assert got[:om + 1] == want


def test_join_group_walk(kc, join):
    # the sub-wavefront group kernels (width > 1) skip wide roots the same way
    want, dags = join
    for width in (4, 32):
        assert kc.count(dags[kc.ORDER_DEGREE], 4, scheme=kc.SCHEME_VC, width=width) == want[4], width


@pytest.mark.parametrize("n", [1100, 2100])
def test_complete_graphs(kc, complete, n):
    # rows of 35 and 66 words: one and two words per lane
    d = complete[n]
    assert d.d_max == n - 1
    for scheme in (1, 2):
        assert kc.count(d, 3, pivot=False, scheme=scheme) == math.comb(n, 3), scheme
        for k in (5, 12):
            assert kc.count(d, k, pivot=True, scheme=scheme) == math.comb(n, k), (scheme, k)


def test_complete_count_all_overflows(kc, complete):
    # C(1100, 550) needs far more than 128 bits
    st, _, _ = kc.count_all_status(complete[1100], pivot=True)
    assert st == kc.EOVERFLOW


def test_cocktail_party(kc):
    m = 600
    d = kc.orient(kc.to_device(synth.complete_multipartite((2,) * m)), kc.ORDER_DEGREE)
    assert d.d_max > kc.MAX_DMAX
    for scheme in (1, 2):
        for k in (3, 4):
            assert kc.count(d, k, pivot=False, scheme=scheme) == math.comb(m, k) * 2 ** k, (scheme, k)


def test_four_words_per_lane(kc):
    # K_4200: rows of 132 words, four per lane
    n = 4200
    d = kc.orient(kc.to_device(synth.complete(n)), kc.ORDER_DEGREE)
    assert d.d_max == n - 1
    assert kc.count(d, 3, pivot=False, scheme=kc.SCHEME_VC) == math.comb(n, 3)
    assert kc.count(d, 4, pivot=True, scheme=kc.SCHEME_VC) == math.comb(n, 4)


@pytest.mark.parametrize("pivot", [False, True])
def test_cancel_flag(kc, join, pivot):
    import torch
    want, dags = join
    f = torch.ones(1, dtype=torch.int32, device="cuda")
    st, _ = kc.count_status(dags[kc.ORDER_DEGREE], 5, pivot, kc.SCHEME_VC, cancel=f.data_ptr())
    assert st == kc.ECANCELED
    f.zero_()
    st, got = kc.count_status(dags[kc.ORDER_DEGREE], 5, pivot, kc.SCHEME_VC, cancel=f.data_ptr())
    assert st == kc.OK and got == want[5]
