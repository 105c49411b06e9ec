"""Seeded generators: determinism and canonical CSR form."""
import numpy as np

import oracle
import synth


def test_er_deterministic_and_canonical():
    a = synth.erdos_renyi(500, 0.03, 7)
    b = synth.erdos_renyi(500, 0.03, 7)
    c = synth.erdos_renyi(500, 0.03, 8)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.row_ptr, b.row_ptr)
    assert not np.array_equal(a.col, c.col)
    assert oracle.validate(a)
    # mean edge count within 5 sigma of C(n,2) p
    mu = 500 * 499 / 2 * 0.03
    assert abs(a.m - mu) < 5 * np.sqrt(mu)


def test_chung_lu_expected_degrees():
    g = synth.chung_lu(20000, 2.1, 20.0, 141.0, 3)
    assert oracle.validate(g)
    assert abs(2 * g.m / g.n - 20.0) < 1.5
    assert g.degrees().max() < 3 * 141


def test_communities_and_dense_core():
    pairs, sizes = synth.communities_pairs(2000, 5, 20, 30, 0.9, 1)
    assert len(sizes) == 5 and sizes.min() >= 20 and sizes.max() <= 30
    expect = sum(s * (s - 1) / 2 for s in sizes) * 0.9
    assert abs(len(pairs) - expect) < 5 * np.sqrt(expect)
    g = synth.dense_core(3000, 10.0, 2.1, 4, 15, 25, 0.9, 5)
    assert oracle.validate(g)


def test_structured_graphs():
    assert synth.complete(6).m == 15
    assert synth.complete_multipartite((2, 3)).m == 6
    assert synth.cycle(7).m == 7
    j = synth.join(synth.complete(3), synth.empty(2))
    assert j.m == 3 + 6
    u = synth.disjoint_union(synth.complete(3), synth.complete(4))
    assert u.m == 3 + 6 and u.n == 7
