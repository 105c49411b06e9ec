"""Writes the power-law workload's clique counts, counted by the oracle.

    python tests/golden/make_powerlaw_counts.py                 # w_max = sqrt(sum w), k = 3..10
    python tests/golden/make_powerlaw_counts.py --wmax 20000 --ks 3,4

The graph is synth.config_powerlaw(): Chung-Lu, n = 1,000,000, mean degree 32,
degree exponent 2.1, seed 2, expected degrees capped at w_max.  It is oriented
by the oracle's degeneracy order (Sec. 3.1) and counted with the oracle's plain
recursion of Fig. 2 over edge roots (Sec. 3.2).  Edge roots are independent, so
they are split into chunks counted in parallel host processes and the per-chunk
counts are summed; every chunk's count is an exact integer.  Besides c_k the file
records the oracle's tree-node count per k (intersections with an adjacency
list, one per l-clique for l = 3 .. k-1) as a cross-check of the sums.

Calls only synth/ and oracle/.
"""
import argparse
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

_DAG = None


def _work(task):
    k, roots = task
    t = time.time()
    c, nodes = oracle.count(_DAG, k, False, oracle.EC, roots=roots, with_nodes=True)
    return k, c, nodes, time.time() - t


def main():
    global _DAG
    ap = argparse.ArgumentParser()
    ap.add_argument("--wmax", type=float, default=0.0, help="0 = sqrt(n x mean) (the Chung-Lu bound)")
    ap.add_argument("--ks", default="3,4,5,6,7,8,9,10")
    ap.add_argument("--chunks", type=int, default=512)
    ap.add_argument("--procs", type=int, default=len(os.sched_getaffinity(0)))
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    n, mean = 1_000_000, 32.0
    wmax = a.wmax if a.wmax > 0 else math.sqrt(n * mean)
    ks = [int(x) for x in a.ks.split(",")]
    t0 = time.time()
    g = synth.config_powerlaw(n=n, wmax=wmax)
    _DAG = oracle.orient(g, oracle.DEGENERACY)
    print("graph n=%d m=%d degeneracy=%d (%.1f s)" % (g.n, g.m, _DAG.degeneracy, time.time() - t0),
          flush=True)
    perm = np.random.default_rng(12345).permutation(_DAG.m).astype(np.int64)
    chunks = np.array_split(perm, a.chunks)
    tasks = [(k, ch) for k in sorted(ks, reverse=True) for ch in chunks]
    tot = {k: 0 for k in ks}
    nodes = {k: 0 for k in ks}
    done = 0
    with mp.get_context("fork").Pool(a.procs) as pool:
        for k, c, nd, dt in pool.imap_unordered(_work, tasks):
            tot[k] += c
            nodes[k] += nd
            done += 1
            if done % 64 == 0 or done == len(tasks):
                print("%d/%d tasks (%.0f s)" % (done, len(tasks), time.time() - t0), flush=True)
    dt = time.time() - t0
    out = a.out or os.path.join(
        HERE, "powerlaw_counts.txt" if a.wmax <= 0 else "powerlaw_wmax%d_counts.txt" % int(wmax))
    with open(out, "w") as f:
        f.write("# Power-law workload: synth.config_powerlaw(wmax=%.6g) = Chung-Lu, n=%d,\n" % (wmax, n))
        f.write("# mean degree 32, degree exponent 2.1, w_max = %.6g, seed 2.\n" % wmax)
        f.write("# Counted by the oracle: degeneracy orientation, plain recursion (Fig. 2), edge\n")
        f.write("# roots (Sec. 3.2), split over %d host processes; %.0f s wall.\n" % (a.procs, dt))
        f.write("# 'c k value' is c_k; 'nodes k value' the oracle's tree nodes at that k.\n")
        f.write("n %d\nm %d\ndegeneracy %d\nd_max %d\n" % (g.n, g.m, _DAG.degeneracy, _DAG.d_max))
        for k in sorted(ks):
            f.write("c %d %d\n" % (k, tot[k]))
        for k in sorted(ks):
            f.write("nodes %d %d\n" % (k, nodes[k]))
    print("wrote", out, {k: tot[k] for k in sorted(ks)}, "in %.1f s" % dt, flush=True)


if __name__ == "__main__":
    main()
