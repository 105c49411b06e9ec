"""Serving (kc_server): every result is the same alone and in the mix, memory
admission refuses oversized queries, and results arrive for every ticket."""
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pool(kc):
    graphs = [synth.chung_lu(3000, 2.1, 12.0, 190.0, 30 + i) for i in range(3)]
    graphs += [synth.dense_core(4000, 8.0, 2.1, 3, 30, 60, 0.8, 40 + i) for i in range(2)]
    graphs += [synth.erdos_renyi(1500, 0.02, 50)]
    dags = [kc.orient(kc.to_device(g), kc.ORDER_DEGENERACY) for g in graphs]
    return graphs, dags


def test_results_same_alone_and_in_mix(kc, pool):
    graphs, dags = pool
    queries = [(g, k, piv) for g in range(len(graphs)) for k in (3, 4, 5, 6, 7) for piv in (False, True)]
    alone = {q: kc.count(dags[q[0]], q[1], pivot=q[2]) for q in queries}
    for g, gr in enumerate(graphs):                     # anchor to the oracle too
        d = oracle.orient(gr, oracle.DEGENERACY)
        for k in (3, 5, 7):
            assert alone[(g, k, False)] == oracle.count(d, k, True, oracle.VC)
    with kc.Server(dags, slots=6, mem_budget=2 << 30) as sv:
        tickets = [(q, sv.submit(*q)) for q in queries * 3]
        for q, t in tickets:
            r = sv.wait(t)
            assert r.status == kc.OK and r.value == alone[q], q
            assert r.t_submit <= r.t_start <= r.t_done


def test_memory_admission(kc, pool):
    graphs, dags = pool
    need = kc.count_workspace_bytes(dags[0], 5, False)
    # an arena smaller than one query's workspace refuses it; one that fits a
    # single query serialises them but still answers every ticket
    with kc.Server(dags, slots=4, mem_budget=max(need // 2, 8192)) as sv:
        r = sv.wait(sv.submit(0, 5))
        assert r.status == kc.ENOMEM
    with kc.Server(dags[:1], slots=4, mem_budget=need + 4096) as sv:
        want = kc.count(dags[0], 5)
        ts = [sv.submit(0, 5) for _ in range(6)]
        rs = [sv.wait(t) for t in ts]
        assert all(r.status == kc.OK and r.value == want for r in rs)
        # one at a time: no two runs overlap
        spans = sorted((r.t_start, r.t_done) for r in rs)
        assert all(spans[i][1] <= spans[i + 1][0] + 1e-3 for i in range(len(spans) - 1))


def test_lds_admission(kc, pool):
    import torch
    graphs, dags = pool
    # every query reports its estimated resident LDS.  A non-pivot count on a
    # graph with 10,000 vertex roots and rows of 8 words (d_max 142) launches a
    # full grid of lane-walk wavefronts of about 14 KB each: it claims more than
    # half the device's LDS, so such queries run one at a time even with free
    # slots and memory; a tiny graph's query claims a small fraction.
    lds_dev = torch.cuda.get_device_properties(0).multi_processor_count * 160 * 1024
    big = kc.orient(kc.to_device(synth.dense_core(10000, 8.0, 2.1, 2, 150, 180, 0.9, 7)), kc.ORDER_DEGENERACY)
    assert 128 < big.d_max <= 256
    tiny = kc.orient(kc.to_device(synth.erdos_renyi(40, 0.3, 1)), kc.ORDER_DEGREE)
    want = kc.count(big, 5)
    with kc.Server([big, tiny], slots=4, mem_budget=4 << 30) as sv:
        rs = [sv.wait(t) for t in [sv.submit(0, 5) for _ in range(4)]]
        small = sv.wait(sv.submit(1, 3))
    assert all(r.status == kc.OK and r.value == want for r in rs)
    assert all(2 * r.lds > lds_dev for r in rs)
    assert small.status == kc.OK and 0 < small.lds < lds_dev // 100
    spans = sorted((r.t_start, r.t_done) for r in rs)
    assert all(spans[i][1] <= spans[i + 1][0] + 1e-3 for i in range(len(spans) - 1))
