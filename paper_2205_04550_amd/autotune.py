"""Autotuner of the batched box-restricted scan's launch shape.

The shape (z-planes per LDS slab, block size, database entries per tile, queries
per chunk) changes only speed, never the result. The tuner times db_query_batch on
the caller's own workload for each candidate with HIP events (median of `reps`
replays) and keeps the fastest.
"""
from __future__ import annotations

import torch


def candidates(nz: int, nq: int):
    """(slab_planes, block_threads, tile_entries, query_chunk) shapes to time."""
    planes = sorted({p for p in (0, 4, 8) if p <= nz})
    chunks = sorted({c for c in (0, 128, 512) if c == 0 or c < max(nq, 129)})
    return [(p, t, tile, c) for p in planes for t in (512, 1024) for tile in (4, 8)
            for c in chunks]


def tune_batch(db, labels: torch.Tensor, rois, k: int, reps: int = 3, configs=None, log=None):
    """Pick the launch shape for this database and query batch.

    Returns (best, table) with table = [(planes, threads, tile, chunk, median_ms), ...];
    the best shape is left applied to `db`.
    """
    nq = labels.shape[0]
    out = (torch.empty((nq, k), dtype=torch.int32, device=labels.device),
           torch.empty((nq, k), dtype=torch.float64, device=labels.device),
           None)
    ws = db.workspace(nq, k)
    table = []
    for cfg in configs or candidates(db.dims[2], nq):
        planes, threads, tile, chunk = (tuple(cfg) + (0, 0))[:4]
        db.tune_batch(planes, threads, tile, chunk)
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
        table.append((planes, threads, tile, chunk, ms))
        if log:
            log(f"  slab planes {planes or 'max'} x {threads} threads, tile {tile or 4}, "
                f"query chunk {chunk or 256}: {ms:.2f} ms")
    best = min(table, key=lambda t: t[-1])
    db.tune_batch(*best[:4])
    return best, table
