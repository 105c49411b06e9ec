"""kc_count_noalloc (the library's fixed device scratch, no allocation) against
kc_count (caller workspace) through the C ABI: identical counts on two calls in
a row, the second on a smaller graph, and the size limit."""
import math

import pytest

import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _cases(d):
    cases = [(3, False, 2), (4, False, 1), (5, False, 2), (7, False, 2), (8, False, 1)]
    if d.d_max <= 64:   # pivot workspaces of wider DAGs exceed the fixed scratch
        cases += [(4, True, 1), (6, True, 2)]
    return cases


def test_noalloc_matches_count_on_consecutive_calls(kc):
    import torch
    torch.cuda.set_device(0)
    big = synth.chung_lu(30000, 2.1, 16.0, math.sqrt(16.0 * 30000), 7)
    small = synth.erdos_renyi(700, 0.03, 8)
    assert small.m < big.m
    for g in (big, small):
        d = kc.orient(kc.to_device(g, DEV), kc.ORDER_DEGENERACY)
        print("noalloc: n=%d m=%d d_max=%d" % (g.n, g.m, d.d_max), flush=True)
        for k, pivot, scheme in _cases(d):
            want = kc.count(d, k, pivot, scheme)
            st, got = kc.count_noalloc_status(d, k, pivot, scheme)
            assert st == kc.OK, (g.n, k, pivot, scheme, kc.strerror(st))
            assert got == want, (g.n, k, pivot, scheme, got, want)


def test_noalloc_refuses_graphs_beyond_the_scratch(kc):
    import torch
    torch.cuda.set_device(0)
    g = synth.chung_lu(300000, 2.1, 32.0, math.sqrt(32.0 * 300000), 9)
    d = kc.orient(kc.to_device(g, DEV), kc.ORDER_DEGENERACY)
    assert kc.count_workspace_bytes(d, 4, False) > 64 << 20
    st, _ = kc.count_noalloc_status(d, 4, False)
    assert st == kc.ENOMEM
    # a graph that fits still counts after the refusal
    s = synth.erdos_renyi(500, 0.05, 3)
    ds = kc.orient(kc.to_device(s, DEV), kc.ORDER_DEGREE)
    assert kc.count_noalloc(ds, 4) == kc.count(ds, 4)
