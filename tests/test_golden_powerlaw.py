"""The power-law count fixtures (tests/golden/powerlaw_counts.txt and
powerlaw_wmax20000_counts.txt) against what fixes them apart from the run that
wrote them: the generator reproduces n and m; the tree-node counts the oracle
recorded separately equal the sums of the stored counts (one node per l-clique,
l = 3 .. k-1, Fig. 2 over edge roots); and c_3, c_4 recomputed on the CPU with
vertex roots under degree order (another root scheme and another orientation)
equal the stored values."""
import math

import pytest

import oracle
import synth
from conftest import load_counts

N, MEAN = 1_000_000, 32.0


@pytest.mark.parametrize("name,wmax", [("powerlaw_counts.txt", math.sqrt(N * MEAN)),
                                       ("powerlaw_wmax20000_counts.txt", 20000.0)])
def test_powerlaw_fixture(name, wmax):
    head, c, nodes = load_counts(name)
    ks = sorted(c)
    for k in ks:
        if all(j in c for j in range(3, k)):
            assert nodes[k] == sum(c[j] for j in range(3, k)), k
    g = synth.config_powerlaw(n=N, wmax=wmax)
    assert (g.n, g.m) == (head["n"], head["m"])
    d = oracle.orient(g, oracle.DEGREE)
    for k in (3, 4):
        assert oracle.count(d, k, False, oracle.VC) == c[k], k
