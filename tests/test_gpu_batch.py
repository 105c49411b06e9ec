"""Batched per-graph counts (kc_batch_count) against the CPU oracle per graph,
against per-graph GPU calls, and across HIP-graph replays."""
import os

import numpy as np
import pytest

import oracle
import synth
from conftest import ROOT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    b = synth.batch(60, seed=11, nmin=20, nmax=400, dmin=4.0, dmax=40.0)
    want = {}
    for g in range(b.ngraphs):
        d = oracle.orient(b.graph(g), oracle.DEGENERACY)
        c, _ = oracle.count_all(d, True, oracle.VC, cap=12)
        want[g] = c
    return b, want


def test_batch_counts_match_oracle(kc, small):
    b, want = small
    bd = kc.batch_to_device(b)
    for k in range(1, 9):
        got = kc.batch_count(bd, k)
        assert got == [want[g][k] for g in range(b.ngraphs)], k


def test_batch_plans_agree(kc, small):
    b, want = small
    bd = kc.batch_to_device(b)
    plans = [kc.BatchPlan.make([(1 << 30, kc.SCHEME_EC)]),
             kc.BatchPlan.make([(100, kc.SCHEME_VC), (250, kc.SCHEME_EC), (1 << 30, kc.SCHEME_VC)])]
    # traversal widths: sub-wavefront groups of every size, alone and mixed with
    # the lane walk across buckets and schemes
    plans += [kc.BatchPlan.make([(1 << 30, sc, wd)]) for sc in (kc.SCHEME_VC, kc.SCHEME_EC)
              for wd in (2, 4, 8, 16, 32)]
    plans.append(kc.BatchPlan.make([(100, kc.SCHEME_VC, 0), (200, kc.SCHEME_EC, 4), (300, kc.SCHEME_VC, 16),
                                    (1 << 30, kc.SCHEME_EC, 0)]))
    for plan in plans:
        for k in (3, 5, 7):
            assert kc.batch_count(bd, k, plan) == [want[g][k] for g in range(b.ngraphs)], (plan.as_list(), k)


def test_batch_plan_rejects_bad_width(kc, small):
    b, _ = small
    bd = kc.batch_to_device(b)
    for wd in (3, 64, -2):
        with pytest.raises(kc.KcError):
            kc.batch_count(bd, 4, kc.BatchPlan.make([(1 << 30, kc.SCHEME_VC, wd)]))


def test_batch_dense_graphs(kc):
    # wide roots (several bitset words) and deep trees (pair tasks) inside a batch
    graphs = [synth.dense_core(3000, 8.0, 2.1, 2, 90, 140, 0.5, 20 + i) for i in range(3)]
    graphs.append(synth.complete(70))
    voff = np.cumsum([0] + [g.n for g in graphs]).astype(np.int32)
    rows, cols, e = [np.zeros(1, np.int64)], [], 0
    for g, a in zip(graphs, voff[:-1]):
        rows.append(g.row_ptr[1:].astype(np.int64) + e)
        cols.append(g.col.astype(np.int64) + a)
        e += g.nnz
    b = synth.Batch(voff, np.concatenate(rows).astype(np.int32), np.concatenate(cols).astype(np.int32))
    bd = kc.batch_to_device(b)
    for k in (4, 6, 7):
        want = [oracle.count(oracle.orient(g, oracle.DEGENERACY), k, True, oracle.VC) for g in graphs]
        for plan in (None, kc.BatchPlan.make([(1 << 30, kc.SCHEME_EC)]),
                     kc.BatchPlan.make([(1 << 30, kc.SCHEME_VC, 8)]), kc.BatchPlan.make([(1 << 30, kc.SCHEME_EC, 32)])):
            assert kc.batch_count(bd, k, plan) == want, (k, plan.as_list() if plan else None)


def test_batch_graph_replay(kc, small):
    import torch
    b, want = small
    bd = kc.batch_to_device(b)
    bg = kc.BatchGraph(bd, 5)
    ref = [want[g][5] for g in range(b.ngraphs)]
    for i in range(4):
        bg.out.fill_(-1)                     # eager work between replays
        bg.replay()
        assert bg.counts() == ref, i
        x = torch.randn(1000, device="cuda").sum().item()
        assert x == x


def load_batch_fixture():
    head, counts = {}, []
    with open(os.path.join(ROOT, "tests", "golden", "batch_counts_k5.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "g":
                assert int(parts[1]) == len(counts)
                counts.append(int(parts[2]))
            else:
                head[parts[0]] = int(parts[1])
    return head, counts


def test_full_batch_matches_oracle_fixture(kc):
    # the batched workload at full size (10,000 graphs, ~1.8e8 edges, Chung-Lu
    # hubs of degree > 1024 whose out-degrees stay within the bitset limit)
    # against the oracle's per-graph counts, with the autotuner-style plans
    head, want = load_batch_fixture()
    b = synth.batch(head["ngraphs"], seed=4)
    assert (b.n, b.nnz) == (head["n"], head["nnz"])
    bd = kc.batch_to_device(b)
    assert bd.max_degree > kc.MAX_DMAX
    for plan in (None, kc.BatchPlan.make([(200, kc.SCHEME_VC), (1000, kc.SCHEME_EC), (1 << 30, kc.SCHEME_VC)]),
                 kc.BatchPlan.make([(200, kc.SCHEME_VC, 4), (1000, kc.SCHEME_VC, 0), (1 << 30, kc.SCHEME_EC, 16)])):
        got = kc.batch_count(bd, head["k"], plan)
        bad = [g for g in range(len(want)) if got[g] != want[g]]
        assert not bad, (plan.as_list() if plan else None, bad[:10])
