"""Writes densecore_count_all.txt: every c_k of the dense-core workload, counted
by the oracle (pivoting, count-all; Sec. 2.3).  Calls only synth/ and oracle/.

    python tests/golden/make_densecore_counts.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    t0 = time.time()
    g = synth.config_densecore()
    d = oracle.orient(g, oracle.DEGENERACY)
    counts, omega = oracle.count_all(d, True, oracle.VC, 1024)
    dt = time.time() - t0
    out = os.path.join(HERE, "densecore_count_all.txt")
    with open(out, "w") as f:
        f.write("# Dense-core workload: synth.config_densecore() = Chung-Lu background n=500000,\n")
        f.write("# mean degree 40, exponent 2.1, w_max = 1000, seed 3, plus 50 planted\n")
        f.write("# communities of U[60, 80] vertices at intra-density 0.9 (seed 4).\n")
        f.write("# Counted by the oracle: degeneracy orientation, pivoting, count-all (Sec. 2.3);\n")
        f.write("# c_0 = 1 is the empty clique.  Written by make_densecore_counts.py in %.0f s.\n" % dt)
        f.write("n %d\nm %d\nomega %d\n" % (g.n, g.m, omega))
        for k, c in enumerate(counts[:omega + 1]):
            f.write("c %d %d\n" % (k, c))
    print("wrote", out, "omega", omega, "in %.1f s" % dt)


if __name__ == "__main__":
    main()
