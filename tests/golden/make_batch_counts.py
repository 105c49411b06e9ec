"""Writes batch_counts_k5.txt: the 5-clique count of every graph of the batched
workload (synth.batch(10000, seed=4): n log-uniform on [50, 5000], half
Erdos-Renyi and half Chung-Lu with degree exponent 2.3 and w_max = n - 1, mean
degree uniform on [8, 64]), counted by the oracle graph by graph (degree
orientation, plain recursion of Fig. 2 over vertex roots), split over host
processes.  Calls only synth/ and oracle/.

    python tests/golden/make_batch_counts.py
"""
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

NGRAPHS, SEED, K = 10000, 4, 5
_B = None


def _work(gs):
    return [(g, oracle.count(oracle.orient(_B.graph(g), oracle.DEGREE), K, False, oracle.VC)) for g in gs]


def main():
    global _B
    t0 = time.time()
    _B = synth.batch(NGRAPHS, seed=SEED)
    chunks = [list(range(i, NGRAPHS, 64)) for i in range(64)]
    out = {}
    with mp.get_context("fork").Pool(len(os.sched_getaffinity(0))) as pool:
        for part in pool.imap_unordered(_work, chunks):
            out.update(part)
    dt = time.time() - t0
    path = os.path.join(HERE, "batch_counts_k5.txt")
    with open(path, "w") as f:
        f.write("# Batched workload synth.batch(%d, seed=%d): per-graph 5-clique counts by the\n" % (NGRAPHS, SEED))
        f.write("# oracle (degree orientation, Fig. 2 over vertex roots); %.0f s wall.\n" % dt)
        f.write("# 'g index count' per graph, in graph order.\n")
        f.write("ngraphs %d\nn %d\nnnz %d\nk %d\n" % (_B.ngraphs, _B.n, _B.nnz, K))
        for g in range(NGRAPHS):
            f.write("g %d %d\n" % (g, out[g]))
    print("wrote", path, "total", sum(out.values()), "in %.1f s" % dt)


if __name__ == "__main__":
    main()
