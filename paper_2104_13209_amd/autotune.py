"""Autotuner for batched counting: root scheme and traversal width per
graph-size bucket.

Graphs of a batch are grouped into size buckets (by vertex count).  For each
bucket, a sample of its graphs is packed into a sub-batch and timed with every
candidate (root scheme, traversal) pair: vertex or edge roots (Sec. 3.2), and
the lane walk or sub-wavefront groups of 4 or 16 lanes (Sec. 3.5)
(kc_batch_count, HIP-event timing after a warm-up call); the fastest pair wins.
Sec. 4.5's guidelines (vertex roots and small groups for small graphs and small
k) are the default order of the candidates, which decides ties.  The resulting
plan can be saved as JSON and loaded later, keyed by the bucket bounds.
"""
from __future__ import annotations

import json

import numpy as np
import torch

from . import SCHEME_EC, SCHEME_VC, BatchPlan, batch_count_async, batch_to_device, batch_workspace_bytes

DEFAULT_BOUNDS = (200, 1000, 1 << 30)
WIDTHS = (0, 4, 16)   # lane walk, groups of 4 and 16 lanes


def _sub_batch(b, graphs):
    """Host sub-batch (voff, row_ptr, col) of the listed graphs of host batch b."""
    voff = [0]
    rows, cols = [np.zeros(1, np.int64)], []
    base_e = 0
    for g in graphs:
        a, z = int(b.voff[g]), int(b.voff[g + 1])
        ea, ez = int(b.row_ptr[a]), int(b.row_ptr[z])
        rp = b.row_ptr[a + 1:z + 1].astype(np.int64) - ea + base_e
        rows.append(rp)
        cols.append(b.col[ea:ez].astype(np.int64) - a + voff[-1])
        base_e += ez - ea
        voff.append(voff[-1] + (z - a))

    class _B:
        pass
    sb = _B()
    sb.voff = np.asarray(voff, np.int32)
    sb.row_ptr = np.concatenate(rows).astype(np.int32)
    sb.col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    return sb


def _time_plan(bd, k, plan, reps=3):
    ws = torch.empty(max(batch_workspace_bytes(bd, k), 1), dtype=torch.uint8, device=bd.row_ptr.device)
    out = torch.empty(2 * bd.ngraphs, dtype=torch.int64, device=bd.row_ptr.device)
    batch_count_async(bd, k, out, ws, plan)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        batch_count_async(bd, k, out, ws, plan)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(b, k, bounds=DEFAULT_BOUNDS, sample=400, seed=0, widths=WIDTHS):
    """Plan for host batch b at clique size k; returns (BatchPlan, report dict)."""
    sizes = np.diff(b.voff.astype(np.int64))
    rng = np.random.default_rng(seed)
    buckets, report = [], []
    lo = 0
    for hi in bounds:
        members = np.nonzero((sizes > lo) & (sizes <= hi))[0]
        if members.size == 0:
            buckets.append((hi, SCHEME_VC, 0))
            lo = hi
            continue
        pick = np.sort(rng.choice(members, size=min(sample, members.size), replace=False))
        bd = batch_to_device(_sub_batch(b, pick))
        t = {}
        for sc in (SCHEME_VC, SCHEME_EC):
            for wd in widths:
                t[(sc, wd)] = _time_plan(bd, k, BatchPlan.make([(1 << 30, sc, wd)]))
        best = min(t, key=t.get)
        buckets.append((hi, best[0], best[1]))
        report.append({"n_hi": int(hi), "graphs": int(members.size), "sampled": int(pick.size),
                       "ms": {("VC" if sc == SCHEME_VC else "EC") + ("_lane" if wd == 0 else "_g%d" % wd):
                              round(v, 3) for (sc, wd), v in t.items()},
                       "scheme": "VC" if best[0] == SCHEME_VC else "EC",
                       "width": int(best[1])})
        lo = hi
    return BatchPlan.make(buckets), report


def save(plan: BatchPlan, path: str, k: int, report=None):
    with open(path, "w") as f:
        json.dump({"k": k, "buckets": plan.as_list(), "report": report or []}, f, indent=1)


def load(path: str) -> BatchPlan:
    with open(path) as f:
        return BatchPlan.make([tuple(x) for x in json.load(f)["buckets"]])
