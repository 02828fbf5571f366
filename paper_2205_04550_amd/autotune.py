"""Autotuner of the batched box-restricted scan's launch shape.

The shape (z-planes per LDS slab, block size) changes only speed, never the
result. The tuner times db_query_batch on the caller's own workload for each
candidate with HIP events (median of `reps` replays) and keeps the fastest.
"""
from __future__ import annotations

import torch


def candidates(nz: int):
    planes = sorted({p for p in (0, 2, 4, 8) if p <= nz})
    return [(p, t) for p in planes for t in (512, 1024)]


def tune_batch(db, labels: torch.Tensor, rois, k: int, reps: int = 3, configs=None, log=None):
    """Pick (slab_planes, block_threads) for this database and query batch.

    Returns (best, table) with table = [(planes, threads, median_ms), ...]; the
    best shape is left applied to `db`.
    """
    nq = labels.shape[0]
    out = (torch.empty((nq, k), dtype=torch.int32, device=labels.device),
           torch.empty((nq, k), dtype=torch.float64, device=labels.device),
           None)
    ws = db.workspace(nq, k)
    table = []
    for planes, threads in configs or candidates(db.dims[2]):
        db.tune_batch(planes, threads)
        db.query_batch(labels, rois, k, out=out, ws=ws)       # records the graph
        times = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            db.query_batch(labels, rois, k, out=out, ws=ws)
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b))
        ms = sorted(times)[len(times) // 2]
        table.append((planes, threads, ms))
        if log:
            log(f"  slab planes {planes or 'max'} x {threads} threads: {ms:.2f} ms")
    best = min(table, key=lambda t: t[2])
    db.tune_batch(best[0], best[1])
    return best, table
