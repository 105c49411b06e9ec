"""The batched workload's count fixture (tests/golden/batch_counts_k5.txt)
against what fixes it apart from the run that wrote it: the generator
reproduces the batch's sizes; graphs of at most 64 vertices match the
brute-force enumerator; a sample of the others matches the oracle's pivoting
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
    small = [g for g in range(b.ngraphs) if b.graph(g).n <= 64]
    assert small
    for g in small[:40]:
        assert oracle.brute_counts(b.graph(g))[5] == c[g], g
    for g in range(0, b.ngraphs, 397):
        d = oracle.orient(b.graph(g), oracle.DEGENERACY)
        assert oracle.count(d, 5, True, oracle.VC) == c[g], g
