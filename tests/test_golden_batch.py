"""The batched workload's count fixture (tests/golden/batch_counts_k5.txt)
against what fixes it apart from the run that wrote it: the generator
reproduces the batch's sizes; graphs of at most 64 vertices and edge density
at most 1/2 match the brute-force enumerator (denser ones hold too many cliques
to enumerate one by one); a sample of the others matches the oracle's pivoting
recursion (Fig. 3) under degeneracy order, where the fixture used the plain
recursion under degree order."""
import os

import oracle
import synth
from conftest import ROOT


def load():
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


def test_batch_fixture():
    head, c = load()
    assert len(c) == head["ngraphs"] == 10000 and head["k"] == 5
    b = synth.batch(head["ngraphs"], seed=4)
    assert (b.n, b.nnz) == (head["n"], head["nnz"])
    small = []
    for g in range(b.ngraphs):
        n, m = b.graph(g).n, b.graph(g).nnz // 2
        if n <= 64 and 4 * m <= n * (n - 1):
            small.append(g)
    assert len(small) >= 40
    for g in small[:40]:
        assert oracle.brute_counts(b.graph(g))[5] == c[g], g
    for g in range(0, b.ngraphs, 397):
        d = oracle.orient(b.graph(g), oracle.DEGENERACY)
        assert oracle.count(d, 5, True, oracle.VC) == c[g], g
