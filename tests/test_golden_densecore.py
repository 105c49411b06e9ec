"""The dense-core count fixture (tests/golden/densecore_count_all.txt) against
what fixes it independently of the pivot recursion that wrote it: the generator
reproduces its n and m, c_1 = n and c_2 = m, and the oracle's plain (non-pivot)
recursion of Fig. 2 gives the same c_3 and c_4."""
import os

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def load():
    head, counts = {}, {}
    with open(os.path.join(HERE, "golden", "densecore_count_all.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "c":
                counts[int(parts[1])] = int(parts[2])
            else:
                head[parts[0]] = int(parts[1])
    return head, counts


def test_densecore_fixture():
    head, c = load()
    g = synth.config_densecore()
    assert (g.n, g.m) == (head["n"], head["m"])
    assert c[0] == 1 and c[1] == g.n and c[2] == g.m
    assert sorted(c) == list(range(head["omega"] + 1)) and c[head["omega"]] > 0
    d = oracle.orient(g, oracle.DEGENERACY)
    assert oracle.count(d, 3, False, oracle.EC) == c[3]
    assert oracle.count(d, 4, False, oracle.EC) == c[4]
