#!/usr/bin/env python3
"""Benchmark of the exact retrieval scan on one MI355X.

Workload (default): the full exact-scan configuration — 50,000 synthetic
tumour simulations on a 128^3 grid, thresholded at 0.25 / 0.675 into FLAIR /
T1Gd masks and bit-packed (26.2 GB resident in HBM), one noisy patient-like
query, exact top-10 by Dice_T1Gd + Dice_FLAIR. One step = one full query:
pack the query, AND+popcount scan of every entry, Dice + score, top-10.
The database build (threshold + pack of the float volumes) is done once
before timing, as the paper's preprocessing is (Sec. 2.3). The line also
carries an "embed" object: the embedding half of the metric (queries/s at a
stated recall@10 against the exact scan) measured in the same run.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Integer VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (lane-ops/s).
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
# Sources of the dominant kernel: committed traffic counters are void once these change.
SCAN_SOURCES = ("paper_2205_04550_amd/csrc/scan.hip", "paper_2205_04550_amd/csrc/common.hpp")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=["full", "small", "batch", "embed", "embed500k", "train", "ds",
                             "sparse"],
                    default="full",
                    help="full: 50,000 x 128^3 exact scan, 1 query (the headline); small: "
                         "1,000 x 64^3; batch: 256 box-restricted queries per launch; embed: "
                         "1,024 held-out queries through encoder + BF16 MFMA distances + "
                         "top-100 + exact rerank; train: encoder training steps (batch 32); "
                         "ds: the exact query on 64^3 / 32^3 order-0 downsampled copies "
                         "(the paper's DS64 / DS32) with Top-N accuracy against 128^3; "
                         "sparse: the exact query over the rows of both row boxes only, and the "
                         "centre-of-mass prefilter with exact rerank; embed500k: FP8 latent "
                         "search over 500,000 simulations generated and encoded in chunks")
    ap.add_argument("--train-steps", type=int, default=300,
                    help="encoder training steps before the embed workload")
    ap.add_argument("--embed-nq", type=int, default=1024)
    ap.add_argument("--embed-streams", type=int, default=2,
                    help="the embedding batch in this many parts, each chain on its own stream")
    ap.add_argument("--nq", type=int, default=256, help="queries per launch (batch workload)")
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target duration of the CPU-oracle sample (0 disables it)")
    ap.add_argument("--build-chunk", type=int, default=2048)
    ap.add_argument("--no-embed", action="store_true",
                    help="full workload only: skip the embedding-search object of the line")
    ap.add_argument("--copy-calibration", type=float, default=0,
                    help="only run a device-to-device copy of this many bytes (3 times), as the "
                         "reference for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE, and exit")
    return ap.parse_args()


def copy_calibration(nbytes: int) -> int:
    import torch
    n = int(nbytes) // 16 * 16
    src = torch.empty(n, dtype=torch.uint8, device="cuda").view(torch.int64)
    src.random_()
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n, "copies": 3}), flush=True)
    return 0


def source_sha(*rel: str) -> str:
    h = hashlib.sha256()
    for r in rel:
        with open(os.path.join(ROOT, r), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


# Committed counter files per workload and the sources of the kernel they measured.
TRAFFIC_FILES = {
    "full": ("scan_full_traffic.json", SCAN_SOURCES),
    "embed": ("pack_pool_query_traffic.json", ("paper_2205_04550_amd/csrc/pack.hip",
                                               "paper_2205_04550_amd/csrc/common.hpp",
                                               "paper_2205_04550_amd/csrc/internal.hpp")),
    "embed500k": ("knn_fp8_500k_traffic.json", ("paper_2205_04550_amd/csrc/knn.hip",
                                                 "paper_2205_04550_amd/csrc/embed_core.hpp",
                                                 "paper_2205_04550_amd/csrc/common.hpp",
                                                 "paper_2205_04550_amd/csrc/embed.hip")),
}


def load_traffic(workload: str):
    """HBM traffic per launch from committed rocprofv3 counter runs, if still current."""
    if workload not in TRAFFIC_FILES:
        return None
    name, sources = TRAFFIC_FILES[workload]
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != source_sha(*sources):
        return None
    return t.get("bytes_per_launch")


def host_info(threads: int) -> dict:
    """What the CPU baseline ran on: threads used, the process's cores, the CPU model."""
    import oracle
    return {"cores": threads, "host_cores": oracle.host_cores(), "cpu_count": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"), "cpu_model": oracle.cpu_model()}


def cpu_baseline(gen, q, t_lo, t_hi, target_s: float):
    """The oracle's for-loop on a bounded sample of the same database: every thread the
    oracle uses on this host, then one thread."""
    import oracle
    threads = oracle._threads()
    n_s = 256
    conc = gen.conc_cpu(0, n_s, threads)            # generation is not timed
    oracle.scan_block(conc[:8], q, t_lo, t_hi, threads=threads)  # warm

    def rate(th, vols, budget):
        passes, elapsed = 0, 0.0
        t0 = time.perf_counter()
        while elapsed < budget or passes == 0:
            oracle.scan_block(vols, q, t_lo, t_hi, threads=th)
            passes += 1
            elapsed = time.perf_counter() - t0
        return passes * len(vols) * gen.nvox / elapsed, passes, elapsed

    v, passes, elapsed = rate(threads, conc, target_s)
    v1, p1, e1 = rate(1, conc[:16], max(2.0, target_s / 4))
    return {"value": v, "unit": "voxels/s", **host_info(threads), "kind": "oracle",
            "value_1thread": v1,
            "sample": f"{n_s} of the {gen.nx}^3 database volumes (float32, host RAM), "
                      f"{passes} passes of the plain for-loop, {elapsed:.1f} s; one thread: 16 "
                      f"volumes, {p1} passes, {e1:.1f} s"}


def cpu_baseline_batch(gen, labels, rois, t_lo, t_hi, target_s: float):
    """The oracle's loop with boxes, on a bounded sample: 64 entries x the first queries."""
    import numpy as np
    import oracle
    threads = oracle._threads()
    conc = gen.conc_cpu(0, 64, threads)
    pairs = 0
    t0 = time.perf_counter()
    q = 0
    while time.perf_counter() - t0 < target_s or q == 0:
        oracle.scan_block(conc, labels[q % len(labels)], t_lo, t_hi, roi=rois[q % len(labels)],
                          threads=threads)
        r = rois[q % len(labels)]
        pairs += 64 * int((r[3] - r[0]) * (r[4] - r[1]) * (r[5] - r[2]))
        q += 1
    el = time.perf_counter() - t0
    return {"value": pairs / el, "unit": "voxels/s", **host_info(threads), "kind": "oracle",
            "sample": f"64 of the {gen.nx}^3 database volumes (float32, host RAM) x {q} box-"
                      f"restricted queries, plain for-loop, {el:.1f} s"}


def cpu_baseline_ds(gen, n, q, side, target_s: float):
    """The oracle's DS query on host cores: volumes and query resampled to side^3 by scipy's
    order-0 zoom (the oracle's routine), then the plain loop; queries/s extrapolated from
    the loop's rate to the n-entry database (resampling not timed)."""
    import oracle
    threads = oracle._threads()
    conc = gen.conc_cpu(0, 64, threads)
    ds = oracle.resample_nearest(conc, (side, side, side))
    qd = oracle.resample_nearest(q, (side, side, side))
    import synth
    oracle.scan_block(ds[:4], qd, synth.T_LO, synth.T_HI, threads=threads)
    passes, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < target_s or passes == 0:
        oracle.scan_block(ds, qd, synth.T_LO, synth.T_HI, threads=threads)
        passes += 1
    el = time.perf_counter() - t0
    vox_s = passes * len(ds) * side ** 3 / el
    return {"value": vox_s / (n * side ** 3), "unit": "queries/s", **host_info(threads),
            "kind": "oracle", "voxels_per_s": vox_s,
            "sample": f"64 volumes resampled to {side}^3, {passes} passes of the plain for-loop, "
                      f"{el:.1f} s; queries/s = voxels/s / ({n} x {side}^3)"}


def cpu_baseline_train(model, db, n, batch, target_s: float):
    """The encoder oracle (float64 torch on the CPU) for training: forward, MSE, backward of
    one batch of mean-pooled database entries (no optimiser step), samples/s."""
    import torch

    import oracle
    from oracle import encoder as E
    from paper_2205_04550_amd import nn
    threads = torch.get_num_threads()
    params = {k: p.detach().to("cpu", torch.float64).requires_grad_(True)
              for k, p in model.params.items()}
    idx = torch.arange(batch, dtype=torch.int32, device="cuda")
    x = nn.meanpool_db(db, idx).detach().to("cpu", torch.float64)
    c, s = model.channels[-1], model.grid >> 4
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < target_s or done == 0:
        loss = E.mse(E.decode(params, E.encode(params, x), c, s), x)
        loss.backward()
        done += 1
    el = time.perf_counter() - t0
    return {"value": done * batch / el, "unit": "samples/s", **host_info(threads),
            "kind": "oracle", "sample": f"{done} forward + backward passes of a batch of {batch} "
                                        f"(float64, torch CPU, {threads} threads), {el:.1f} s"}


def roi_work(rois, n: int):
    """Voxel pairs compared and packed word positions (both masks) inside the boxes."""
    vox = 0
    words = 0
    for x0, y0, z0, x1, y1, z1 in rois.tolist():
        vox += (x1 - x0) * (y1 - y0) * (z1 - z0)
        words += (((x1 - 1) >> 5) - (x0 >> 5) + 1) * (y1 - y0) * (z1 - z0)
    return vox * n, 2 * words * n


def executed_batch_ops(db, rois, n: int, tile: int = 4) -> float:
    """Integer VALU ops of one batched launch over the rows it scans: per query and tile of
    `tile` entries, the box rows clipped to the union of the tile members' row boxes, times
    the box's words per row, 2 masks, the members and 3 ops (measurement bookkeeping)."""
    import torch
    order = db.tile_order[:n].to(torch.int64)
    b = db.boxes[:n].to(torch.int64)[order]
    pad = (-n) % tile
    if pad:
        b = torch.cat([b, b[-1:].expand(pad, 4)])
    t = b.view(-1, tile, 4)
    empty = ~((t[..., 1] > t[..., 0]) & (t[..., 3] > t[..., 2]))
    big, small = 1 << 30, -(1 << 30)
    uz0 = torch.where(empty, big, t[..., 0]).amin(1)
    uz1 = torch.where(empty, small, t[..., 1]).amax(1)
    uy0 = torch.where(empty, big, t[..., 2]).amin(1)
    uy1 = torch.where(empty, small, t[..., 3]).amax(1)
    total = 0
    for x0, y0, z0, x1, y1, z1 in rois.tolist():
        dz = (torch.clamp(uz1, max=z1) - torch.clamp(uz0, min=z0)).clamp(min=0)
        dy = (torch.clamp(uy1, max=y1) - torch.clamp(uy0, min=y0)).clamp(min=0)
        nw = ((x1 - 1) >> 5) - (x0 >> 5) + 1
        total += int((dz * dy).sum()) * nw
    return float(total) * 2 * tile * 3


def bench_batch(args, db, gen, n, build_s) -> int:
    """256 noisy queries, each cut to its own box, per db_query_batch launch."""
    import numpy as np
    import torch

    import oracle
    import synth
    t_lo, t_hi, k, nq = synth.T_LO, synth.T_HI, args.k, args.nq
    log(f"making {nq} queries and boxes")
    labels, srcs = synth.make_queries(gen, n, nq, synth.BATCH_QUERY_SEED)
    rois = synth.make_rois(labels, synth.ROI_SEED)
    lab_d = torch.from_numpy(labels).cuda()
    out = (torch.empty((nq, k), dtype=torch.int32, device="cuda"),
           torch.empty((nq, k), dtype=torch.float64, device="cuda"),
           torch.empty((nq, k, 6), dtype=torch.int32, device="cuda"))
    ws = db.workspace(nq, k)
    db.query_batch(lab_d, rois, k, out=out, ws=ws)
    db.sync()
    # Re-check two queries' returned entries with the oracle.
    ok = True
    for qi in (0, nq - 1):
        idx = out[0][qi].cpu().numpy().tolist()
        _, o_cnt, o_sc = oracle.scan(gen, n, labels[qi], t_lo, t_hi, roi=rois[qi], indices=idx)
        ok &= bool(np.array_equal(o_sc.view(np.uint64), out[1][qi].cpu().numpy().view(np.uint64))
                   and np.array_equal(out[2][qi].cpu().numpy().view(np.uint32).astype(np.uint64),
                                      o_cnt))
    log(f"returned entries of queries 0 and {nq - 1} re-checked by the oracle: "
        f"{'ok' if ok else 'MISMATCH'}")
    from paper_2205_04550_amd import autotune
    log("autotuning the launch shape (z-planes per LDS slab x block size x entries per tile x "
        "queries per chunk)")
    best, table = autotune.tune_batch(db, lab_d, rois, k, reps=3, log=log)
    log(f"picked {best[0] or 'max'} planes x {best[1]} threads, tile {best[2] or 4}, chunk "
        f"{best[3] or 256} ({best[4]:.2f} ms)")
    for _ in range(args.warmup):
        db.query_batch(lab_d, rois, k, out=out, ws=ws)
    torch.cuda.synchronize()
    db.profile(True)
    db.profile_read()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        db.query_batch(lab_d, rois, k, out=out, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g_ms, launches = db.profile_read()
    db.profile(False)
    ms = (t1 - t0) * 1e3 / args.steps
    pairs_vox, words = roi_work(rois, n)
    g_avg = g_ms / max(1, launches)
    dense_ops = 3 * words   # per packed word and mask: AND, popcount-add (I), popcount-add (B)
    ops = executed_batch_ops(db, rois, n, best[2] or 4)
    achieved = ops / (g_avg * 1e-3)
    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline_batch(gen, labels, rois, t_lo, t_hi, args.cpu_seconds)
        log(f"cpu oracle {cpu['value']:.3e} voxel pairs/s on {cpu['cores']} threads")
    log(f"{ms:.2f} ms per {nq}-query launch; {pairs_vox / (ms * 1e-3):.3e} voxel pairs/s; "
        f"{achieved / VALU_PEAK_OPS:.1%} of integer VALU issue")
    line = {
        "metric": "database voxels compared/sec",
        "value": pairs_vox / (ms * 1e-3),
        "unit": "voxels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"batched exact scan, {nq} box-restricted queries x {n} sims x "
                               f"{gen.nx}^3, top-{k} each, one kernel launch (a block per tile of "
                               f"entries and query chunk, costliest tiles first) from a HIP graph",
                   "n_db": n, "nq": nq, "k": k, "mean_box_voxels": pairs_vox / n / nq},
        "queries_per_s": nq / (ms * 1e-3),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s", "frac": achieved / VALU_PEAK_OPS, "traffic": None,
                     "kernel": "batch_lds_kernel (from a HIP graph)",
                     "kernel_avg_ms": g_avg,
                     "algorithmic_ops_per_launch": ops,
                     "dense_box_ops_per_launch": dense_ops,
                     "note": "ops over the rows of each box clipped to the union of the tile's "
                             "row boxes, the rows the kernel scans; the dense count treats every "
                             "box row of every entry as work",
                     "hbm_floor_gb_per_launch": n * 2 * gen.nvox / 8 / 1e9},
        "autotune": {"picked": {"slab_planes": best[0], "block_threads": best[1],
                                "tile_entries": best[2], "query_chunk": best[3]},
                     "table_columns": ["slab_planes", "block_threads", "tile_entries",
                                       "query_chunk", "median_ms"],
                     "table_ms": [list(t) for t in table]},
        "cpu_baseline": cpu,
        "parity": {"returned_entries_rechecked_by_oracle": ok},
        "build_s": build_s,
    }
    print(json.dumps(line), flush=True)
    return 0 if ok else 1


# MI355X vector FP32 without packed instructions (which are not used: 157.3 TFLOP/s is the
# packed-FP32 figure): 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz.
FP32_VECTOR_PEAK = 78.6e12
FP32_MFMA_PEAK = 157.3e12        # MI355X dense FP32 matrix FLOP/s
BF16_MFMA_PEAK = 2.5e15          # MI355X dense BF16 matrix FLOP/s
FP8_MFMA_PEAK = 5.0e15           # MI355X dense FP8 matrix FLOP/s


def model_macs(model) -> int:
    """Multiply-accumulates of one forward pass of the autoencoder for one sample."""
    g, c = model.grid, model.channels
    macs = 0
    for i in range(4):
        out = (g >> (i + 1)) ** 3
        macs += out * c[i + 1] * c[i] * 27          # encoder convolution i
        macs += out * c[i + 1] * c[i] * 27          # its mirrored transposed convolution
    macs += 2 * model.flat * model.latent           # encoder and decoder linear layers
    return macs


def train_encoder(model, db, n: int, steps: int, batch: int, seed: int = 7, mask=None):
    import torch
    from paper_2205_04550_amd import nn
    opt = nn.Adam(model, lr=1e-3)
    g = torch.Generator().manual_seed(seed)
    losses = []
    for _ in range(steps):
        idx = torch.randint(0, n, (batch,), generator=g).to(torch.int32).cuda()
        losses.append(nn.train_step(model, opt, nn.meanpool_db(db, idx, mask=mask)))
    return opt, [float(l) for l in losses]


def bench_train(args, db, gen, n, build_s) -> int:
    """Encoder training: batch 32 of mean-pooled 2 x 64^3 inputs; forward, backward, Adam."""
    import torch
    from paper_2205_04550_amd import nn
    batch = 32
    model = nn.AutoEncoder(grid=gen.nx // 2, latent=512, seed=0)
    opt = nn.Adam(model, lr=1e-3)
    g = torch.Generator().manual_seed(7)
    idx_all = [torch.randint(0, n, (batch,), generator=g).to(torch.int32).cuda()
               for _ in range(args.warmup + args.steps)]
    losses = []
    for i in range(args.warmup):
        losses.append(nn.train_step(model, opt, nn.meanpool_db(db, idx_all[i])))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        losses.append(nn.train_step(model, opt, nn.meanpool_db(db, idx_all[args.warmup + i])))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    flop = 3 * 2 * model_macs(model) * batch    # forward + backward (about twice the forward)
    losses = [float(l) for l in losses]
    log(f"{ms:.2f} ms per training step of {batch}; loss {losses[0]:.5f} -> {losses[-1]:.5f}")
    line = {
        "metric": "encoder training samples/sec", "value": batch / (ms * 1e-3),
        "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (bf16 weights)", "data": "synthetic",
        "config": {"workload": f"autoencoder training, batch {batch} x 2 x {model.grid}^3, "
                               f"latent 512, {model.n_params()} parameters, Adam",
                   "n_db": n},
        "roofline": {"bound": "alu", "achieved": flop / (ms * 1e-3) / 1e12,
                     "peak": FP32_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": flop / (ms * 1e-3) / FP32_VECTOR_PEAK, "traffic": None,
                     "kernel": "whole step (forward convolutions and linear layers on the FP32 "
                               "matrix cores, backward kernels on the vector ALUs)",
                     "note": "peak = the vector FP32 rate without packed instructions",
                     "algorithmic_flop_per_step": flop},
        "loss_first_last": [losses[0], losses[-1]],
        "cpu_baseline": (cpu_baseline_train(model, db, n, batch, args.cpu_seconds)
                         if args.cpu_seconds > 0 else None),
        "build_s": build_s,
    }
    print(json.dumps(line), flush=True)
    return 0


def small_latency(db, qd, k, out, ws, reps: int = 50, flush_bytes: int = 1 << 30) -> dict:
    """Single-query latency of the exact scan on a database that fits the caches: warm
    (back to back), cold (after writing flush_bytes, which evicts the L2s and the 256 MB
    Infinity Cache), and as one replay of a captured HIP graph (checked against the eager
    result). Medians of per-query HIP event times, in microseconds."""
    import numpy as np
    import torch

    cur = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(f):
        e0.record()
        f()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e3

    q = lambda: db.query(qd, k, out=out, ws=ws)
    for _ in range(5):
        q()
    warm = [timed(q) for _ in range(reps)]
    flush = torch.empty(flush_bytes // 4, dtype=torch.int32, device="cuda")
    cold = []
    for i in range(reps // 2):
        flush.fill_(i)
        torch.cuda.synchronize()
        cold.append(timed(q))
    del flush
    want = [t.clone() for t in out if t is not None]
    side = torch.cuda.Stream()
    side.wait_stream(cur)
    with torch.cuda.stream(side):
        q()
    cur.wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        q()
    for t in out:
        if t is not None:
            t.zero_()
    graph = [timed(g.replay) for _ in range(reps)]
    same = all(torch.equal(a, b) for a, b in zip([t for t in out if t is not None], want))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    back_to_back = (time.perf_counter() - t0) * 1e6 / reps
    med = lambda v: float(np.median(v))
    log(f"latency: warm {med(warm):.1f} us, cold {med(cold):.1f} us, graph replay {med(graph):.1f} us "
        f"({back_to_back:.1f} us back to back); graph result equals eager: {same}")
    return {"warm_us": med(warm), "cold_us": med(cold), "graph_replay_us": med(graph),
            "graph_back_to_back_us": back_to_back, "graph_equals_eager": same,
            "flush_bytes": flush_bytes, "reps": reps,
            "note": "per query: pack + scan + top-k; cold after writing flush_bytes; medians of "
                    "HIP event times"}


def cpu_baseline_embed(model, X, labels, gen, n, n_cand, k, target_s: float):
    """The oracle's embedding query on host cores, one query at a time: float64 mean-pool
    and encoder, float64 direct distances to the stored latents, top-n_cand, and the
    for-loop Dice on the candidates (their volumes regenerated on the CPU)."""
    import numpy as np
    import torch

    import oracle
    from oracle import encoder as E
    threads = oracle._threads()
    # The encoder as the GPU runs it: bfloat16 working weights, float biases, activations
    # stored as bfloat16 between the convolutions.
    params = {k2: (model.work[k2] if k2 in model.work else p).detach().to("cpu", torch.float64)
              for k2, p in model.params.items()}
    xlat = E.bf16_decode(X.codes.view(torch.int16).cpu().numpy())
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < target_s or done == 0:
        lab = labels[done % len(labels)]
        z = E.encode_bf16_activations(params, torch.from_numpy(E.meanpool(lab[None]))).numpy()
        d = E.sqdist_direct(z, xlat)[0]
        cand = E.topk_by_distance(d[None], n_cand)[0]
        _, cnt, sc = oracle.scan(gen, n, lab, synth_t()[0], synth_t()[1], indices=cand.tolist(),
                                 threads=threads)
        oracle.rank(sc, k)
        done += 1
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "queries/s", **host_info(threads), "kind": "oracle",
            "sample": f"{done} of the held-out queries, one at a time (encoder, float64 "
                      f"distances to {n} latents, top-{n_cand}, for-loop Dice), {el:.1f} s"}


def synth_t():
    import synth
    return synth.T_LO, synth.T_HI


HASH_GAMMA = 3.0   # weight of the Bi-half layer's pull of latents towards their codes
VAE_BETA = 1e-5    # KL weight against the per-voxel mean MSE (about 2.6 against a voxel sum)


def _query_boxes(lab, gen, bits):
    """Row boxes (z0, z1, y0, y1) [nq] of the rows of labels lab [nq][nz][ny][nx] holding one
    of `bits`."""
    import torch
    rows = ((lab & bits).reshape(lab.shape[0], gen.nz, gen.ny, gen.nx).amax(dim=3) != 0)
    zany, yany = rows.any(dim=2), rows.any(dim=1)
    ar_z = torch.arange(gen.nz, device=lab.device)
    ar_y = torch.arange(gen.ny, device=lab.device)
    big = 1 << 20
    return (torch.where(zany, ar_z, big).amin(1), torch.where(zany, ar_z + 1, -big).amax(1),
            torch.where(yany, ar_y, big).amin(1), torch.where(yany, ar_y + 1, -big).amax(1))


def _plane_rows(eb, zr, q, gen, rb, lines):
    """Per (query, entry): rows one plane's scan reads, or the 128-byte lines they touch:
    slices of (entry box n query box), in each the entry's y-range of that slice cut to the
    boxes' y-range. eb [..][4] entry boxes, zr [..][nz] the entry's packed slice ranges,
    q = (z0, z1, y0, y1) of the query (broadcast against eb)."""
    import torch
    z0 = torch.maximum(eb[..., 0], q[0])
    z1 = torch.minimum(eb[..., 1], q[1])
    y0 = torch.maximum(eb[..., 2], q[2])
    y1 = torch.minimum(eb[..., 3], q[3])
    zs = torch.arange(gen.nz, device=eb.device)
    inz = (zs >= z0[..., None]) & (zs < z1[..., None])
    a0 = torch.maximum(zr & 0xffff, y0[..., None])
    a1 = torch.minimum(zr >> 16, y1[..., None])
    ok = inz & (a1 > a0)
    if lines:
        n = (a1 * rb + 127) // 128 - (a0 * rb) // 128
    else:
        n = a1 - a0
    return (torch.where(ok, n, torch.zeros_like(n))).sum(dim=-1)


def rerank_bytes(db, lab_d, cand, gen, lines: bool = False, scored=None) -> float:
    """Database bytes the candidate-scoring kernel reads: per (query, candidate) and plane, the
    rows of the slices inside both row boxes of that plane (the boxes of both masks for FLAIR,
    the T1Gd boxes for T1Gd) that lie in the candidate's y-range of that plane in the slice
    (measurement bookkeeping), over the pairs of `scored` (bool [nq][nc]; None: all).
    lines=True counts the 128-byte cache lines those rows touch instead (a slice's run of rows
    starts and ends inside a line)."""
    import torch
    rb = gen.nx // 32 * 4                                          # bytes per row and plane
    c = cand.to(torch.int64)
    total = 0.0
    for p, (bits, boxes) in enumerate(((3, db.boxes), (2, db.tboxes))):
        qz0, qz1, qy0, qy1 = _query_boxes(lab_d, gen, bits)
        q = (qz0[:, None], qz1[:, None], qy0[:, None], qy1[:, None])
        for r0 in range(0, c.shape[0], 128):                      # bounded temporaries
            eb = boxes[c[r0:r0 + 128]].to(torch.int64)            # [128][nc][4]
            zr = db.zranges[c[r0:r0 + 128]][..., p].to(torch.int64)   # [128][nc][nz]
            qq = tuple(t[r0:r0 + 128] for t in q)
            rows = _plane_rows(eb, zr, qq, gen, rb, lines)
            if scored is not None:
                rows = rows * scored[r0:r0 + 128].to(rows.dtype)
            total += float(rows.sum())
    return total * (128 if lines else rb)


def bound_scored(db, lab_d, cand, k, gen):
    """The candidates the bound-ordered rerank scores, by its rule on the host (measurement
    bookkeeping): every candidate's bound (the score formula at the sums over 16^3 blocks of
    the smaller of the two sides' counts), the first n1 = max(16, k) rounded to 16 in (bound
    desc, slot asc) order, then those whose bound reaches the k-th best exact score of the
    first n1. Returns (scored bool [nq][nc], bytes of the bound pass: the candidates' block
    counts and the queries' rows inside their row boxes)."""
    import torch
    nq, nc = cand.shape
    nbx, nby, nbz, nbp = db.block_dims()
    n1 = (max(k, 16) + 15) // 16 * 16
    if nbp == 0 or k <= 0 or n1 > 64 or nc <= n1:
        return torch.ones((nq, nc), dtype=torch.bool, device=cand.device), 0.0
    ws = db.rerank_workspace(nq)
    db.rerank_pack(lab_d, ws)
    db.set_rerank_bound(False)
    fi, fs, _ = db.rerank_packed(ws, cand, nc)                     # every candidate's score
    db.set_rerank_bound(True)
    c = cand.to(torch.int64)
    _, perm = torch.sort(c, dim=1)
    fsort, fperm = torch.sort(fi.to(torch.int64), dim=1)
    sc = torch.empty_like(fs).scatter_(1, perm, fs.gather(1, fperm))   # exact score per slot
    nz, ny, nx = gen.nz, gen.ny, gen.nx
    pad = (0, -nx % 16, 0, -ny % 16, 0, -nz % 16)
    ub = torch.empty((nq, nc), dtype=torch.float64, device=cand.device)
    pc = db.popcounts.to(torch.int64)

    def dice(i, a, b):
        den = a + b
        return torch.where(den == 0, torch.ones_like(i, dtype=torch.float64),
                           (2 * i).to(torch.float64) / den.clamp(min=1).to(torch.float64))

    for r0 in range(0, nq, 64):
        lab = lab_d[r0:r0 + 64]
        qb = []
        for bit in (1, 2):
            m = torch.nn.functional.pad(((lab & bit) != 0).to(torch.int32), pad)
            m = m.reshape(m.shape[0], nbz, 16, nby, 16, nbx, 16).sum(dim=(2, 4, 6))
            qb.append(torch.nn.functional.pad(m.reshape(m.shape[0], -1), (0, nbp - nbx * nby * nbz)))
        qb = torch.stack(qb, dim=1)                                 # [b][2][nbp]
        a = qb.sum(-1).to(torch.int64)                              # query popcounts
        bc = db.block_counts[c[r0:r0 + 64]].to(torch.int32) & 0xffff   # [b][nc][2][nbp]
        u = torch.minimum(bc, qb[:, None]).sum(-1).to(torch.int64)  # [b][nc][2]
        b = pc[c[r0:r0 + 64]]
        ub[r0:r0 + 64] = dice(u[..., 1], a[:, None, 1], b[..., 1]) + dice(u[..., 0], a[:, None, 0],
                                                                        b[..., 0])
    order = torch.sort(-ub, dim=1, stable=True)[1]
    ubs = ub.gather(1, order)
    tau = sc.gather(1, order[:, :n1]).topk(k, dim=1)[0][:, -1:]
    pos = torch.arange(nc, device=cand.device)[None] < n1
    keep = pos | (ubs >= tau)
    scored = torch.zeros_like(keep).scatter_(1, order, keep)
    qz0, qz1, qy0, qy1 = _query_boxes(lab_d, gen, 3)
    qrows = ((qz1 - qz0).clamp(min=0) * (qy1 - qy0).clamp(min=0)).sum()
    bound_bytes = nq * nc * 2 * nbp * 2 + float(qrows) * 2 * (gen.nx // 8)
    return scored, bound_bytes


def encoder_forward_flop(model, nq: int) -> float:
    """FLOP of the encoder's forward pass (convolutions and linear layer) for nq samples."""
    g, c = model.grid, model.channels
    macs = sum((g >> (i + 1)) ** 3 * c[i + 1] * c[i] * 27 for i in range(4))
    macs += model.flat * model.latent
    return 2.0 * macs * nq


def encode_stage_bytes(model, gen, nq: int) -> float:
    """HBM bytes of the embedding step's encode stage for nq queries (BF16 forward): the
    labels read once (by the query packing), the packed masks and the pooled counts written,
    the counts read by the first two layers (one kernel: the first layer's output stays on
    chip), the second layer's output written and read once (bfloat16), the third and fourth
    layers in one kernel (the third's output stays on chip), the fourth's output (float)
    written and read once and the latents written."""
    g, c = model.grid, model.channels
    per = gen.nvox + 2 * gen.nvox // 8 + 2 * gen.nvox // 8
    per += 2 * 2 * (g >> 2) ** 3 * c[2]
    per += 2 * 4 * (g >> 4) ** 3 * c[4] + 4 * model.latent
    return float(per) * nq


def embed_run(args, db, gen, n, with_variants: bool) -> dict:
    """Held-out queries through the encoder, the fused latent search (distances + top-100 in
    one pass) and the exact rerank. Returns the measurements as a dict."""
    import numpy as np
    import torch

    import synth
    from paper_2205_04550_amd import binding as B, nn
    nq, n_cand, k = args.embed_nq, 100, 15
    model = nn.AutoEncoder(grid=gen.nx // 2, latent=512, seed=0)
    log(f"training the encoder for {args.train_steps} steps of 32")
    t0 = time.perf_counter()
    _, losses = train_encoder(model, db, n, args.train_steps, 32)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    log(f"trained in {train_s:.1f} s, loss {losses[0]:.5f} -> {losses[-1]:.5f}")
    t0 = time.perf_counter()
    lat = torch.empty((n, model.latent), dtype=torch.float32, device="cuda")
    dims = (gen.nx, gen.ny, gen.nz)
    for s in range(0, n, 500):
        idx = torch.arange(s, min(n, s + 500), dtype=torch.int32, device="cuda")
        lat[s:s + idx.numel()] = model.encode_planes_bf16(db.planes, dims, idx)
    X = B.Latents(lat, B.EMB_BF16)
    torch.cuda.synchronize()
    encode_db_s = time.perf_counter() - t0
    log(f"encoded {n} entries in {encode_db_s:.1f} s; making {nq} held-out queries")
    labels, _ = synth.make_queries(gen, n, nq, synth.HELDOUT_SEED, held_out_seed=synth.HELDOUT_SEED)
    lab_d = torch.from_numpy(labels).cuda()
    lab_host_sample = labels[:32].copy()
    del labels
    # Exact top-k of every query (the ground truth), one exact scan per query.
    ws1 = db.workspace(1, k)
    ex_idx = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    ex_out = (torch.empty(k, dtype=torch.int32, device="cuda"),
              torch.empty(k, dtype=torch.float64, device="cuda"), None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in range(nq):
        db.query(lab_d[q], k, out=ex_out, ws=ws1)
        ex_idx[q].copy_(ex_out[0])
    torch.cuda.synchronize()
    exact_ms_per_query = (time.perf_counter() - t0) * 1e3 / nq
    log(f"exact scan: {exact_ms_per_query:.3f} ms per query")

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    stage = np.zeros(3)
    pack_ms = 0.0

    # One read of the query labels: the rerank's packing also writes their pooled counts,
    # which the encoder's first layer reads instead of the labels.
    ws_rr = db.rerank_workspace(nq)
    pooled = torch.empty((nq, gen.nz // 2, gen.ny // 2, gen.nx // 2), dtype=torch.uint8,
                         device="cuda")
    kws = B.knn_workspace(nq, n, n_cand)
    kout = (torch.empty((nq, n_cand), dtype=torch.int32, device="cuda"),
            torch.empty((nq, n_cand), dtype=torch.float32, device="cuda"))

    def step(timed: bool):
        if timed:
            ev[0].record()
        db.rerank_pack_pool(lab_d, ws_rr, pooled)
        if timed:
            ev[4].record()
        ql = model.encode_counts_bf16(pooled)
        Q = B.Latents(ql, B.EMB_BF16)
        if timed:
            ev[1].record()
        ci, cd = B.emb_knn(Q, X, n_cand, direct=True, ws=kws, out=kout)
        if timed:
            ev[2].record()
        out = db.rerank_packed(ws_rr, ci, k)
        if timed:
            ev[3].record()
        return out, ci

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    db.profile(True)
    db.profile_read()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        (idx, score, counts), ci = step(True)
        torch.cuda.synchronize()
        stage += [ev[i].elapsed_time(ev[i + 1]) for i in range(3)]
        pack_ms += ev[0].elapsed_time(ev[4])
    t1 = time.perf_counter()
    rr_ms, rr_launches = db.profile_read()
    db.profile(False)
    rr_avg = rr_ms / max(1, rr_launches)
    # The same batch in H parts, each chain (packing, encoder, search, rerank) on a stream of
    # its own, so that one part's memory-bound kernels run beside another's compute-bound ones;
    # the top k must equal the one-stream step's.
    H = max(1, args.embed_streams)
    halves = []
    for h in range(H):
        a, b = h * nq // H, (h + 1) * nq // H
        halves.append({"lab": lab_d[a:b], "ws": db.rerank_workspace(b - a),
                       "pooled": torch.empty((b - a, gen.nz // 2, gen.ny // 2, gen.nx // 2),
                                             dtype=torch.uint8, device="cuda"),
                       "kws": B.knn_workspace(b - a, n, n_cand),
                       "kout": (torch.empty((b - a, n_cand), dtype=torch.int32, device="cuda"),
                                torch.empty((b - a, n_cand), dtype=torch.float32, device="cuda")),
                       "stream": torch.cuda.Stream()})

    def step_halves():
        cur = torch.cuda.current_stream()
        outs = []
        for hh in halves:
            hh["stream"].wait_stream(cur)
            with torch.cuda.stream(hh["stream"]):
                db.rerank_pack_pool(hh["lab"], hh["ws"], hh["pooled"])
                Qh = B.Latents(model.encode_counts_bf16(hh["pooled"]), B.EMB_BF16)
                ch, _ = B.emb_knn(Qh, X, n_cand, direct=True, ws=hh["kws"], out=hh["kout"])
                outs.append(db.rerank_packed(hh["ws"], ch, k))
        for hh in halves:
            cur.wait_stream(hh["stream"])
        return outs

    for _ in range(args.warmup):
        step_halves()
    torch.cuda.synchronize()
    th0 = time.perf_counter()
    for _ in range(args.steps):
        outs = step_halves()
    torch.cuda.synchronize()
    ms_halves = (time.perf_counter() - th0) * 1e3 / args.steps
    halves_equal = bool(torch.equal(torch.cat([o[0] for o in outs]), idx) and
                        torch.equal(torch.cat([o[1] for o in outs]).view(torch.int64),
                                    score.view(torch.int64)))
    log(f"{H} parts on {H} streams: {ms_halves:.3f} ms per {nq} queries "
        f"({nq / (ms_halves * 1e-3):.0f} q/s), top-k equal to one stream: {halves_equal}")
    scored, bound_bytes = bound_scored(db, lab_d, ci, k, gen)
    rr_bytes = rerank_bytes(db, lab_d, ci, gen, scored=scored) + bound_bytes
    n_scored = float(scored.double().sum(1).mean())
    rr_roof = {"bound": "hbm", "achieved": rr_bytes / (rr_avg * 1e-3) / 1e9,
               "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": rr_bytes / (rr_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
               "kernel": "query_block_kernel + rerank_ub_kernel + rerank_order_kernel + rerank_score_kernel<4> x 2 + rerank_gate_kernel",
               "kernel_avg_ms": rr_avg, "algorithmic_bytes_per_launch": rr_bytes,
               "candidates_scored_per_query": n_scored,
               "note": "the rerank's scoring between HIP events; bytes = every candidate's "
                       "16^3-block counts and the query's rows inside its row box (the bound), "
                       "then for the candidates scored: database rows of the slices inside "
                       "(query row box n candidate row box) for FLAIR, inside (query T1Gd row "
                       "box n candidate T1Gd row box) for T1Gd, each within the candidate's "
                       "y-range of that plane in the slice"}
    pack_ms /= args.steps
    pack_bytes = float(gen.nvox + 2 * gen.nvox // 8 + gen.nvox // 8) * nq
    pack_roof = {"bound": "hbm", "achieved": pack_bytes / (pack_ms * 1e-3) / 1e9,
                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": pack_bytes / (pack_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "traffic": load_traffic("embed") if nq == 1024 else None,
                 "kernel": "pack_pool_query_kernel + sum_parts_kernel", "kernel_avg_ms": pack_ms,
                 "algorithmic_bytes_per_launch": pack_bytes,
                 "note": "the query packing between HIP events; bytes = the labels read once, "
                         "the packed masks and the pooled counts written"}
    ms = (t1 - t0) * 1e3 / args.steps
    stage /= args.steps
    got = idx.cpu().numpy()
    ex = ex_idx.cpu().numpy()
    recall10 = float(np.mean([len(set(got[q, :10]) & set(ex[q, :10])) / 10 for q in range(nq)]))
    top_n = {f"top{t}": float(np.mean([ex[q, 0] in got[q, :t] for q in range(nq)])) for t in (1, 5, 15)}
    cand_recall = float(np.mean([len(set(ci[q].cpu().numpy()) & set(ex[q, :10])) / 10
                                 for q in range(min(nq, 256))]))
    cpu = None
    if args.cpu_seconds > 0:
        log("timing the CPU oracle on a sample of the queries")
        cpu = cpu_baseline_embed(model, X, lab_host_sample, gen, n, n_cand, k, args.cpu_seconds)
        log(f"cpu oracle {cpu['value']:.3f} queries/s on {cpu['cores']} threads")
    gemm_flop = 2.0 * nq * n * model.latent
    enc_flop = encoder_forward_flop(model, nq)
    enc_bytes = encode_stage_bytes(model, gen, nq)
    names = ["pack queries (masks + pooled counts), encode",
             "latent distances + top-100 in one pass (BF16 MFMA), direct-form candidate distances",
             "exact rerank"]
    dom = int(np.argmax(stage))
    # The job's step: the batch in parts on their own streams when that is faster and gives
    # the same top k; the stage times below are the one-stream step's.
    ms_job = ms_halves if H > 1 and halves_equal and ms_halves < ms else ms
    log(f"{ms_job:.2f} ms per {nq} queries ({nq / (ms_job * 1e-3):.0f} q/s; one stream "
        f"{ms:.2f} ms); one-stream stages "
        + ", ".join(f"{a} {b:.3f} ms" for a, b in zip(names, stage))
        + f"; recall@10 {recall10:.3f}; {top_n}; speed-up vs exact "
          f"{exact_ms_per_query * nq / ms_job:.0f}x; rerank scored {n_scored:.1f} of {n_cand} "
          f"candidates per query (query packing {pack_ms:.3f} ms)")
    out = {
        "metric": "queries/sec at recall@10", "value": nq / (ms_job * 1e-3), "unit": "queries/s",
        "ms_per_step": ms_job, "steps": args.steps, "warmup": args.warmup, "dtype": "bf16",
        "config": {"workload": f"embedding search, {nq} held-out queries x {n} latents (512-d "
                               f"BF16), top-{n_cand} by MFMA distance, exact 128^3 Dice rerank, "
                               f"top-{k}", "n_db": n, "nq": nq, "n_cand": n_cand,
                   "train_steps": args.train_steps, "streams": H if ms_job == ms_halves else 1},
        "one_stream_ms_per_step": ms, "parts_streams": H, "parts_ms_per_step": ms_halves,
        "parts_topk_equal_one_stream": halves_equal,
        "recall_at_10": recall10, **top_n, "candidate_recall_at_10": cand_recall,
        "speedup_vs_exact_scan": exact_ms_per_query * nq / ms_job,
        "exact_ms_per_query": exact_ms_per_query,
        "stages_ms": dict(zip(names, stage.tolist())),
        "dominant_stage": names[dom],
        "roofline": pack_roof if pack_ms >= rr_avg else rr_roof,
        "rerank_roofline" if pack_ms >= rr_avg else "pack_roofline":
            rr_roof if pack_ms >= rr_avg else pack_roof,
        "encode_stage_roofline": {
            "bound": "hbm", "achieved": enc_bytes / (stage[0] * 1e-3) / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": enc_bytes / (stage[0] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes": enc_bytes, "stage_ms": stage[0],
            "encoder_flop": enc_flop, "encoder_tflops": enc_flop / (stage[0] * 1e-3) / 1e12,
            "note": "the stage's HBM bytes: the labels read once (the query packing), the "
                    "packed masks and the pooled counts written, the counts read by the first "
                    "two layers (one kernel; the first layer's activations stay on chip), the "
                    "second layer's bfloat16 activations written once and read once by the third "
                    "and fourth layers (one kernel; the third's activations stay on chip), the "
                    "last layer's float output; the convolutions run on the BF16 matrix cores, "
                    "the linear head on the FP32 ones"},
        "latent_search": {"bound": "mfma", "achieved_tflops": gemm_flop / (stage[1] * 1e-3) / 1e12,
                          "peak_tflops": BF16_MFMA_PEAK / 1e12,
                          "frac": gemm_flop / (stage[1] * 1e-3) / BF16_MFMA_PEAK,
                          "kernels": "knn_kernel<false, false> + knn_merge_kernel + "
                                     "knn_direct_kernel<false>", "ms": stage[1],
                          "note": "no distance matrix is written"},
        "cpu_baseline": cpu, "train_s": train_s,
        "encode_db_s": encode_db_s, "train_loss_first_last": [losses[0], losses[-1]],
    }
    if with_variants:
        out["variants"] = embed_variants(args, db, gen, n, model, lat, lab_d, ex, Dbuf_shape=(nq, n))
    return out


def embed_variants(args, db, gen, n, model, lat, lab_d, ex, Dbuf_shape) -> dict:
    """Other codes of the same search: FP8 latents of the encoder, the hashing variant, and
    the paper's two single-mask encoders (plain and variational) with summed L2."""
    import numpy as np
    import torch

    from paper_2205_04550_amd import binding as B, nn
    nq, n_cand, k = args.embed_nq, 100, 15
    dims = (gen.nx, gen.ny, gen.nz)
    Dbuf = torch.empty(Dbuf_shape, dtype=torch.float32, device="cuda")

    def leg(name, fmt, encode_q, Xl):
        for _ in range(max(1, args.warmup)):
            o = db.query_embed(fmt, encode_q(), Xl, lab_d, n_cand, k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            o = db.query_embed(fmt, encode_q(), Xl, lab_d, n_cand, k, out=o)
        torch.cuda.synchronize()
        lms = (time.perf_counter() - t0) * 1e3 / args.steps
        g = o[0].cpu().numpy()
        r = {"ms_per_batch": lms, "queries_per_s": nq / (lms * 1e-3),
             "recall_at_10": float(np.mean([len(set(g[q, :10]) & set(ex[q, :10])) / 10
                                            for q in range(nq)])),
             **{f"top{t}": float(np.mean([ex[q, 0] in g[q, :t] for q in range(nq)]))
                for t in (1, 5, 15)}}
        log(f"{name}: {r['queries_per_s']:.0f} q/s, recall@10 {r['recall_at_10']:.3f}, "
            f"Top-1/5/15 {r['top1']:.3f}/{r['top5']:.3f}/{r['top15']:.3f}")
        return r

    variants = {}
    X8 = B.Latents(lat, B.EMB_FP8)

    def enc_fp8():
        with torch.no_grad():
            return B.Latents(model.encode_labels_bf16(lab_d), B.EMB_FP8)
    variants["fp8_latents"] = leg("FP8 latents", B.EMB_FP8, enc_fp8, X8)
    del X8
    log(f"training the hashing encoder (Bi-half layer) for {args.train_steps} steps of 32")
    model_h = nn.AutoEncoder(grid=gen.nx // 2, latent=512, seed=1, hash_gamma=HASH_GAMMA)
    t0 = time.perf_counter()
    _, losses_h = train_encoder(model_h, db, n, args.train_steps, 32)
    torch.cuda.synchronize()
    hash_train_s = time.perf_counter() - t0
    with torch.no_grad():
        for s0 in range(0, n, 500):
            idx_b = torch.arange(s0, min(n, s0 + 500), dtype=torch.int32, device="cuda")
            lat[s0:s0 + idx_b.numel()] = model_h.encode_planes_bf16(db.planes, dims, idx_b)
    Xh = B.BinaryCodes(lat)

    def enc_hash():
        with torch.no_grad():
            return B.BinaryCodes(model_h.encode_labels_bf16(lab_d), Xh.thr)
    variants["bf_hash_512bit"] = leg("Bi-half codes (Hamming)", B.EMB_BIN, enc_hash, Xh)
    variants["bf_hash_512bit"].update({"train_s": hash_train_s, "gamma": HASH_GAMMA,
                                       "train_loss_first_last": [losses_h[0], losses_h[-1]]})
    del Xh

    # The paper's own formulation: separate T1Gd and FLAIR encoders, distance
    # L2_T1Gd + L2_FLAIR; plain autoencoders and variational ones (search on the mean).
    for tag, kw in (("two_ae_l2sum", {}), ("two_vae_l2sum", {"vae_beta": VAE_BETA})):
        log(f"training two single-mask encoders ({tag}) for {args.train_steps} steps of 32 each")
        t0 = time.perf_counter()
        pair, Xs, rec = [], [], []
        for m in (1, 0):                                  # T1Gd, then FLAIR
            mdl = nn.AutoEncoder(grid=gen.nx // 2, channels=(1, 8, 16, 32, 64), latent=512,
                                 seed=2 + m, **kw)
            _, lm = train_encoder(mdl, db, n, args.train_steps, 32, mask=m)
            rec.append([lm[0], lm[-1]])
            with torch.no_grad():
                for s0 in range(0, n, 500):
                    idx_b = torch.arange(s0, min(n, s0 + 500), dtype=torch.int32, device="cuda")
                    lat[s0:s0 + idx_b.numel()] = mdl.encode_planes_bf16(db.planes, dims, idx_b,
                                                                        mask=m)
            Xs.append(B.Latents(lat, B.EMB_BF16))
            pair.append((mdl, m))
        torch.cuda.synchronize()
        tr_s = time.perf_counter() - t0

        def step_pair():
            with torch.no_grad():
                qs = [B.Latents(mdl.encode_labels_bf16(lab_d, mask=m), B.EMB_BF16)
                      for mdl, m in pair]
            D = B.emb_distances_l2sum(qs[0], Xs[0], qs[1], Xs[1], out=Dbuf)
            ci2, _ = B.emb_topk_min(D, n_cand)
            return db.rerank(lab_d, ci2, k)

        for _ in range(max(1, args.warmup)):
            o = step_pair()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            o = step_pair()
        torch.cuda.synchronize()
        lms = (time.perf_counter() - t0) * 1e3 / args.steps
        g2 = o[0].cpu().numpy()
        r = {"ms_per_batch": lms, "queries_per_s": nq / (lms * 1e-3),
             "recall_at_10": float(np.mean([len(set(g2[q, :10]) & set(ex[q, :10])) / 10
                                            for q in range(nq)])),
             **{f"top{t}": float(np.mean([ex[q, 0] in g2[q, :t] for q in range(nq)]))
                for t in (1, 5, 15)},
             "train_s": tr_s, "recon_loss_first_last_t1gd_flair": rec}
        if "vae_beta" in kw:
            r["beta"] = kw["vae_beta"]
        log(f"{tag}: {r['queries_per_s']:.0f} q/s, recall@10 {r['recall_at_10']:.3f}, "
            f"Top-1/5/15 {r['top1']:.3f}/{r['top5']:.3f}/{r['top15']:.3f}")
        variants[tag] = r
        del Xs, pair

    return variants


def bench_embed(args, db, gen, n, build_s) -> int:
    """Held-out queries through encoder, fused BF16 MFMA latent search and exact rerank, and
    the other codes of the same search."""
    r = embed_run(args, db, gen, n, with_variants=True)
    line = {"metric": r.pop("metric"), "value": r.pop("value"), "unit": r.pop("unit"),
            "n_gpus": 1, "steps": r.pop("steps"), "warmup": r.pop("warmup"),
            "ms_per_step": r.pop("ms_per_step"), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": r.pop("dtype"), "data": "synthetic",
            "config": r.pop("config"), **r, "build_s": build_s}
    print(json.dumps(line), flush=True)
    return 0


def bench_embed500k(args, db, gen, n, build_s, n_big: int = 500_000) -> int:
    """FP8 latent search at 500,000 entries: simulations generated, thresholded, pooled and
    encoded chunk by chunk (their masks are not kept: they would need 262 GB); 1,024
    held-out queries; FP8 MFMA distances + top-100, recall@10 against the BF16 path over
    the same latents (no exact rerank: the masks are gone)."""
    import numpy as np
    import torch

    import synth
    from paper_2205_04550_amd import TumorDB, binding as B, nn
    nq, n_cand = args.embed_nq, 100
    model = nn.AutoEncoder(grid=gen.nx // 2, latent=512, seed=0)
    log(f"training the encoder for {args.train_steps} steps of 32")
    train_encoder(model, db, n, args.train_steps, 32)
    log(f"generating and encoding {n_big} simulations in chunks")
    t0 = time.perf_counter()
    chunk = 2048
    lat = torch.empty((n_big, model.latent), dtype=torch.float32, device="cuda")
    buf = torch.empty((chunk, gen.nvox), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    for s0 in range(0, n_big, chunk):
        c = min(chunk, n_big - s0)
        p = torch.from_numpy(gen.params(s0, c).view(np.float64).reshape(c, 8).copy()).cuda()
        gen.conc_gpu(p.data_ptr(), c, buf.data_ptr(), stream)
        part = TumorDB(gen.nx, gen.ny, gen.nz, c, synth.T_LO, synth.T_HI)
        part.append(buf[:c])
        with torch.no_grad():
            for b0 in range(0, c, 512):
                idx = torch.arange(b0, min(c, b0 + 512), dtype=torch.int32, device="cuda")
                lat[s0 + b0:s0 + b0 + idx.numel()] = model.encode_planes_bf16(
                    part.planes, (gen.nx, gen.ny, gen.nz), idx)
        del part
        if (s0 // chunk) % 40 == 0:
            log(f"  {s0 + c}/{n_big}")
    torch.cuda.synchronize()
    del buf
    torch.cuda.empty_cache()
    gen_s = time.perf_counter() - t0
    X8 = B.Latents(lat, B.EMB_FP8)
    X16 = B.Latents(lat, B.EMB_BF16)
    del lat
    torch.cuda.empty_cache()
    labels, _ = synth.make_queries(gen, n, nq, synth.HELDOUT_SEED, held_out_seed=synth.HELDOUT_SEED)
    lab_d = torch.from_numpy(labels).cuda()
    del labels
    ql = model.encode_labels_bf16(lab_d)
    Q8, Q16 = B.Latents(ql, B.EMB_FP8), B.Latents(ql, B.EMB_BF16)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    kws = B.knn_workspace(nq, n_big, n_cand)

    def run_fused(Q, X):
        ev[0].record()
        ci, _ = B.emb_knn(Q, X, n_cand, direct=True, ws=kws)
        ev[1].record()
        return ci

    def timed(fn, Q, X, two_stage=False):
        for _ in range(max(1, args.warmup)):
            fn(Q, X)
        torch.cuda.synchronize()
        a_ms = b_ms = 0.0
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ci = fn(Q, X)
            torch.cuda.synchronize()
            a_ms += ev[0].elapsed_time(ev[1])
            if two_stage:
                b_ms += ev[1].elapsed_time(ev[2])
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        return ms, a_ms / args.steps, b_ms / args.steps, ci

    res = {}
    for name, Q, X in (("bf16", Q16, X16), ("fp8", Q8, X8)):
        ms, k_ms, _, ci = timed(run_fused, Q, X)
        res[name] = {"ms_per_batch": ms, "emb_knn_ms": k_ms, "cand": ci.cpu().numpy()}
        log(f"{name}: {ms:.3f} ms per {nq} queries (fused distances + top-{n_cand}: "
            f"{k_ms:.3f} ms)")
    # The earlier two-pass path for comparison: the [M][N] distance matrix with group
    # minima, then the top-100 bounded by those minima.
    D = torch.empty((nq, n_big), dtype=torch.float32, device="cuda")
    gws = B.groups_workspace(nq, n_big)

    def run_matrix(Q, X):
        ev[0].record()
        B.emb_distances_groups(Q, X, gws, out=D)
        ev[1].record()
        ci, _ = B.emb_topk_groups(D, n_cand, gws)
        ev[2].record()
        return ci

    ms_m, g_m, s_m, ci_m = timed(run_matrix, Q8, X8, two_stage=True)
    same = bool(np.array_equal(ci_m.cpu().numpy(), res["fp8"]["cand"]))
    log(f"fp8 with the distance matrix: {ms_m:.3f} ms (distances {g_m:.3f}, top-{n_cand} "
        f"{s_m:.3f}); same candidates as the fused path: {same}")
    del D, gws
    res["fp8_distance_matrix_path"] = {"ms_per_batch": ms_m, "distances_ms": g_m,
                                       "select_ms": s_m, "same_candidates": same}
    c8, c16 = res["fp8"].pop("cand"), res["bf16"].pop("cand")
    recall10 = float(np.mean([len(set(c8[q, :10]) & set(c16[q, :10])) / 10 for q in range(nq)]))
    cover = float(np.mean([len(set(c8[q]) & set(c16[q, :10])) / 10 for q in range(nq)]))
    flop = 2.0 * nq * n_big * 512
    k8 = res["fp8"]["emb_knn_ms"]
    log(f"FP8 recall@10 vs BF16 {recall10:.3f}; BF16 top-10 inside FP8 top-{n_cand}: {cover:.3f}")
    cpu = None
    if args.cpu_seconds > 0:
        log("timing the CPU oracle: float64 direct distances to every FP8 latent, top-100")
        cpu = cpu_baseline_latents(Q8, X8, n_cand, args.cpu_seconds)
        log(f"cpu oracle {cpu['value']:.3f} queries/s on {cpu['cores']} threads")
    line = {
        "metric": "queries/sec at recall@10", "value": nq / (res["fp8"]["ms_per_batch"] * 1e-3),
        "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["fp8"]["ms_per_batch"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp8", "data": "synthetic",
        "config": {"workload": f"FP8 latent search, {nq} held-out queries x {n_big} latents (512-d "
                               f"OCP e4m3, per-row scale), top-{n_cand}; recall against BF16 latents",
                   "n_db": n_big, "nq": nq, "n_cand": n_cand},
        "recall_at_10_vs_bf16": recall10, "bf16_top10_within_fp8_top100": cover,
        "paths": res, "generate_and_encode_s": gen_s,
        "roofline": {"bound": "mfma", "achieved": flop / (k8 * 1e-3) / 1e12,
                     "peak": BF16_MFMA_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": flop / (k8 * 1e-3) / BF16_MFMA_PEAK,
                     "traffic": load_traffic("embed500k"),
                     "kernel": "emb_knn: knn_kernel<true, false> + knn_merge_kernel + "
                               "knn_direct_kernel<true>", "kernel_avg_ms": k8,
                     "algorithmic_flop_per_launch": flop,
                     "note": "e4m3 codes decoded exactly to BF16 in LDS and multiplied on the BF16 "
                             "matrix cores (peak 2.5 PFLOP/s); no distance matrix is written; "
                             "time of the whole call (three kernels)"},
        "cpu_baseline": cpu, "build_s": build_s,
    }
    print(json.dumps(line), flush=True)
    return 0


def cpu_baseline_latents(Q, X, n_cand: int, target_s: float):
    """The oracle's latent search on host cores, one query at a time: float64 direct-form
    distances to every stored (dequantised) database latent, then the n_cand smallest."""
    import numpy as np
    import torch

    import oracle
    from oracle import encoder as E
    from paper_2205_04550_amd import binding as B

    def deq(L):
        if L.fmt == B.EMB_BF16:
            return E.bf16_decode(L.codes.view(torch.int16).cpu().numpy())
        return E.e4m3_decode(L.codes.cpu().numpy()) * L.scale.cpu().numpy().astype(np.float64)[:, None]
    x, q = deq(X), deq(Q)
    threads = 1                      # numpy's einsum and sort run on one thread
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < target_s or done == 0:
        d = E.sqdist_direct(q[done % len(q)][None], x)
        E.topk_by_distance(d, n_cand)
        done += 1
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "queries/s", **host_info(threads), "kind": "oracle",
            "sample": f"{done} queries, float64 direct distances to {x.shape[0]} latents and a "
                      f"stable sort, {el:.1f} s (numpy, one thread)"}


def bench_ds(args, db, gen, n, build_s) -> int:
    """DS64 / DS32 (paper Sec. 2.3, Table 2): held-out queries, exact query on downsampled
    copies of database and query; Top-N = share of queries whose 128^3 best match is in
    the downsampled top-N."""
    import numpy as np
    import torch

    import synth
    from paper_2205_04550_amd import TumorDB
    from paper_2205_04550_amd.binding import labels_resample
    nq, k = args.embed_nq, 15
    labels, _ = synth.make_queries(gen, n, nq, synth.HELDOUT_SEED, held_out_seed=synth.HELDOUT_SEED)
    lab_d = torch.from_numpy(labels).cuda()
    del labels
    ws = db.workspace(1, 1)
    out1 = (torch.empty(1, dtype=torch.int32, device="cuda"),
            torch.empty(1, dtype=torch.float64, device="cuda"), None)
    best = np.empty(nq, dtype=np.int64)
    best_score = np.empty(nq)
    for q in range(nq):
        db.query(lab_d[q], 1, out=out1, ws=ws)
        best[q] = int(out1[0].item())
        best_score[q] = float(out1[1].item())
    results = {}
    for side in (gen.nx // 2, gen.nx // 4):
        t0 = time.perf_counter()
        ds = TumorDB(side, side, side, n, db.t_lo, db.t_hi)
        ds.append_resampled(db)
        torch.cuda.synchronize()
        build = time.perf_counter() - t0
        qd = labels_resample(lab_d, (side, side, side))
        wsd = ds.workspace(1, k)
        outk = (torch.empty(k, dtype=torch.int32, device="cuda"),
                torch.empty(k, dtype=torch.float64, device="cuda"), None)
        got = np.empty((nq, k), dtype=np.int64)
        for q in range(min(nq, 8)):
            ds.query(qd[q], k, out=outk, ws=wsd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for q in range(nq):
            ds.query(qd[q], k, out=outk, ws=wsd)
            got[q] = outk[0].cpu().numpy()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / nq
        # Time the queries alone (no host copy per query) for the throughput figure.
        ds.profile(True)
        ds.profile_read()
        t0 = time.perf_counter()
        for q in range(nq):
            ds.query(qd[q], k, out=outk, ws=wsd)
        torch.cuda.synchronize()
        ms_q = (time.perf_counter() - t0) * 1e3 / nq
        scan_ms, launches = ds.profile_read()
        ds.profile(False)
        topn = {f"top{t}": float(np.mean([best[q] in got[q, :t] for q in range(nq)])) for t in (1, 5, 15)}
        alg = n * 2 * side ** 3 // 8
        results[f"DS{side}"] = {"ms_per_query": ms_q, **topn, "build_s": build,
                                "scan_kernel_ms": scan_ms / max(1, launches),
                                "scan_GBps": alg / (scan_ms / max(1, launches) * 1e-3) / 1e9}
        log(f"DS{side}: {ms_q:.3f} ms per query; Top-1/5/15 {topn['top1']:.3f} / {topn['top5']:.3f} / "
            f"{topn['top15']:.3f}")
        del ds
        torch.cuda.empty_cache()
    cpu = None
    if args.cpu_seconds > 0:
        log("timing the CPU oracle on 64^3 copies (order-0 resampling, plain loop)")
        cpu = cpu_baseline_ds(gen, n, lab_d[0].cpu().numpy(), gen.nx // 2, args.cpu_seconds)
        log(f"cpu oracle {cpu['value']:.3f} queries/s on {cpu['cores']} threads")
    line = {
        "metric": "queries/sec at Top-N accuracy", "value": 1e3 / results[f"DS{gen.nx // 2}"]["ms_per_query"],
        "unit": "queries/s", "n_gpus": 1, "steps": nq, "warmup": 8,
        "ms_per_step": results[f"DS{gen.nx // 2}"]["ms_per_query"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"downsampled exact scans (order-0) of {n} x {gen.nx}^3, {nq} held-out "
                               f"queries, Top-N against the {gen.nx}^3 best match", "n_db": n, "nq": nq},
        "results": results, "mean_best_score_128": float(best_score.mean()),
        "roofline": {"bound": "hbm", "achieved": results[f"DS{gen.nx // 2}"]["scan_GBps"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": results[f"DS{gen.nx // 2}"]["scan_GBps"] / HBM_PEAK_GBS,
                     "traffic": None, "kernel": "scan_kernel (64^3 copy)",
                     "kernel_avg_ms": results[f"DS{gen.nx // 2}"]["scan_kernel_ms"]},
        "cpu_baseline": cpu, "build_s": build_s,
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_sparse(args, db, gen, n, build_s) -> int:
    """Exact query reading only the rows inside both row boxes (same results as the
    dense scan, checked here for every timed query), and the centre-of-mass prefilter
    (Sec. 2.3 radiomics query's location step) followed by exact Dice on its candidates."""
    import numpy as np
    import torch

    import synth
    k, nq = args.k, 64
    V = gen.nvox
    labels, _ = synth.make_queries(gen, n, nq, synth.QUERY_SEED)
    lab_d = torch.from_numpy(labels).cuda()
    del labels
    ws = db.workspace(1, k)
    mk = lambda: (torch.empty(k, dtype=torch.int32, device="cuda"),
                  torch.empty(k, dtype=torch.float64, device="cuda"),
                  torch.empty((k, 6), dtype=torch.int32, device="cuda"))
    out_d, out_s = mk(), mk()
    same = True
    for q in range(nq):
        db.query(lab_d[q], k, out=out_d, ws=ws)
        db.query_sparse(lab_d[q], k, out=out_s, ws=ws)
        same &= all(bool(torch.equal(a, b)) for a, b in zip(out_d, out_s))
    torch.cuda.synchronize()
    log(f"sparse == dense on {nq} queries: {same}")
    # Bytes the sparse kernel reads from HBM: per plane, the database rows of the slices where
    # that plane's boxes meet (the boxes of both masks for FLAIR, the T1Gd boxes for T1Gd) that
    # lie in the entry's y-range of that plane in the slice; measurement bookkeeping from the
    # stored boxes and ranges and the query's set rows.
    rb = gen.nx // 32 * 4                              # bytes per row and plane
    rows_read = np.zeros(nq)                           # rows inside both boxes of both masks
    bytes_read, line_bytes = np.zeros(nq), np.zeros(nq)
    eb_any = db.boxes[:n].to(torch.int64)
    for p, (bits, boxes) in enumerate(((3, db.boxes), (2, db.tboxes))):
        eb = boxes[:n].to(torch.int64)
        zr = db.zranges[:n][..., p].to(torch.int64)
        qb = _query_boxes(lab_d, gen, bits)
        for q in range(nq):
            qq = tuple(t[q] for t in qb)
            bytes_read[q] += float(_plane_rows(eb, zr, qq, gen, rb, False).sum()) * rb
            line_bytes[q] += float(_plane_rows(eb, zr, qq, gen, rb, True).sum()) * 128
            if p == 0:
                dz = (torch.minimum(eb_any[:, 1], qq[1]) - torch.maximum(eb_any[:, 0], qq[0])).clamp(min=0)
                dy = (torch.minimum(eb_any[:, 3], qq[3]) - torch.maximum(eb_any[:, 2], qq[2])).clamp(min=0)
                rows_read[q] = float((dz * dy).sum())
    for _ in range(args.warmup):
        for q in range(min(nq, 8)):
            db.query_sparse(lab_d[q], k, out=out_s, ws=ws)
    torch.cuda.synchronize()
    reps = max(1, args.steps // 10)
    db.profile(True)
    db.profile_read()
    t0 = time.perf_counter()
    for _ in range(reps):
        for q in range(nq):
            db.query_sparse(lab_d[q], k, out=out_s, ws=ws)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    scan_ms, launches = db.profile_read()
    db.profile(False)
    ms_q = el * 1e3 / (reps * nq)
    kern_ms = scan_ms / max(1, launches)
    achieved = float(bytes_read.mean()) / (kern_ms * 1e-3) / 1e9
    alg = n * 2 * (V // 8)
    log(f"sparse: {ms_q:.3f} ms/query, kernel {kern_ms:.3f} ms, reads {bytes_read.mean() / 1e9:.2f} GB "
        f"of the dense {alg / 1e9:.2f} GB ({achieved:.0f} GB/s)")

    # Centre-of-mass prefilter + exact rerank over held-out queries.
    nqc, ks = args.embed_nq, 15
    held, _ = synth.make_queries(gen, n, nqc, synth.HELDOUT_SEED, held_out_seed=synth.HELDOUT_SEED)
    held_d = torch.from_numpy(held).cuda()
    del held
    best = np.empty(nqc, dtype=np.int64)
    for q in range(nqc):
        db.query_sparse(held_d[q], 1, out=out_s, ws=ws)
        best[q] = int(out_s[0][0].item())
    com = {}
    for n_cand in (100, 1000):
        o = db.query_com(held_d[:8], n_cand, ks)
        wsc = torch.empty(LIB_ws_com(db, nqc, n_cand), dtype=torch.uint8, device="cuda")
        o = db.query_com(held_d, n_cand, ks, ws=wsc)
        torch.cuda.synchronize()
        db.profile(True)
        db.profile_read()
        t0 = time.perf_counter()
        o = db.query_com(held_d, n_cand, ks, ws=wsc, out=o)
        torch.cuda.synchronize()
        el_c = time.perf_counter() - t0
        rr_ms, rr_n = db.profile_read()
        db.profile(False)
        got = o[0].cpu().numpy()
        topn = {f"top{t}": float(np.mean([best[q] in got[q, :t] for q in range(nqc)]))
                for t in (1, 5, 15)}
        scored, bound_b = bound_scored(db, held_d, o[3], ks, gen)
        rr_alg = rerank_bytes(db, held_d, o[3], gen, scored=scored) + bound_b
        rr_lines = rerank_bytes(db, held_d, o[3], gen, lines=True, scored=scored) + bound_b
        com[f"n_cand_{n_cand}"] = {"queries_per_s": nqc / el_c, "ms_per_query": el_c * 1e3 / nqc,
                                   **topn, "rerank_score_ms": rr_ms / max(1, rr_n),
                                   "rerank_algorithmic_bytes": rr_alg,
                                   "rerank_line_bytes": rr_lines,
                                   "candidates_scored_per_query":
                                       float(scored.double().sum(1).mean()),
                                   "bound_pass_bytes": bound_b}
        log(f"COM prefilter {n_cand}: {nqc / el_c:.0f} q/s, Top-1/5/15 {topn['top1']:.3f} / "
            f"{topn['top5']:.3f} / {topn['top15']:.3f}")
        del wsc
    cpu = None
    if args.cpu_seconds > 0:
        log("timing the CPU oracle sample (the plain loop reads every voxel)")
        q0 = lab_d[0].cpu().numpy()
        cpu = cpu_baseline(gen, q0, synth.T_LO, synth.T_HI, args.cpu_seconds)
        cpu["note"] = ("the oracle's for-loop compares every voxel of the grid; its rate is "
                       "voxels of the whole grid per second")
    vox_read = float(rows_read.mean()) * gen.nx       # voxels in the rows inside both row boxes
    line = {
        "metric": "database voxels compared/sec", "value": vox_read / (ms_q * 1e-3),
        "unit": "voxels/s", "n_gpus": 1, "steps": reps * nq, "warmup": args.warmup,
        "ms_per_step": ms_q, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"exact scan reading only the rows inside both row boxes (the T1Gd "
                               f"plane only inside both T1Gd row boxes), {n} sims x {gen.nx}^3, "
                               f"{nq} noisy-entry queries, top-{k}; value counts the voxels of the "
                               "rows inside both row boxes",
                   "n_db": n, "grid": [gen.nx, gen.ny, gen.nz], "k": k},
        "voxels_read_per_query": vox_read,
        "dense_equivalent_voxels_per_s": n * V / (ms_q * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "box_scan_kernel", "kernel_avg_ms": kern_ms,
                     "bytes_read_per_launch_mean": float(bytes_read.mean()),
                     "line_bytes_per_launch_mean": float(line_bytes.mean()),
                     "dense_algorithmic_bytes_per_launch": alg},
        "parity": {"sparse_equals_dense_on_all_queries": bool(same)},
        "com_prefilter": com, "cpu_baseline": cpu, "build_s": build_s,
    }
    print(json.dumps(line), flush=True)
    return 0 if same else 1


def LIB_ws_com(db, nq, n_cand):
    from paper_2205_04550_amd.binding import LIB
    return LIB.db_query_com_workspace_bytes(db._h, nq, n_cand)


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path runs "
              "on a single MI355X; multi-GPU sharding is a design note only).", file=sys.stderr)
        return 2
    if args.copy_calibration:
        return copy_calibration(int(args.copy_calibration))
    import numpy as np
    import torch

    import synth
    from paper_2205_04550_amd import TumorDB

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    gen, n = (synth.SMALL, synth.SMALL_N) if args.workload == "small" else (synth.FULL, synth.FULL_N)
    t_lo, t_hi, k = synth.T_LO, synth.T_HI, args.k
    V = gen.nvox

    # ---- build the database (not timed: one-off preprocessing) ----
    log(f"building {n} x {gen.nx}^3 database on the GPU")
    tb = time.perf_counter()
    db = TumorDB(gen.nx, gen.ny, gen.nz, n, t_lo, t_hi)
    chunk = min(args.build_chunk, n)
    buf = torch.empty((chunk, V), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        p = torch.from_numpy(gen.params(s, c).view(np.float64).reshape(c, 8).copy()).cuda()
        gen.conc_gpu(p.data_ptr(), c, buf.data_ptr(), stream)
        db.append(buf[:c])
    torch.cuda.synchronize()
    del buf
    torch.cuda.empty_cache()
    build_s = time.perf_counter() - tb
    log(f"built in {build_s:.1f} s")

    if args.workload == "batch":
        return bench_batch(args, db, gen, n, build_s)
    if args.workload == "train":
        return bench_train(args, db, gen, n, build_s)
    if args.workload == "embed":
        return bench_embed(args, db, gen, n, build_s)
    if args.workload == "ds":
        return bench_ds(args, db, gen, n, build_s)
    if args.workload == "sparse":
        return bench_sparse(args, db, gen, n, build_s)
    if args.workload == "embed500k":
        return bench_embed500k(args, db, gen, n, build_s)

    src = synth.query_source(n, synth.QUERY_SEED, 0)
    q = gen.query(src, t_lo, t_hi, synth.QUERY_SEED, 0)
    qd = torch.from_numpy(q).cuda()
    out = (torch.empty(k, dtype=torch.int32, device="cuda"),
           torch.empty(k, dtype=torch.float64, device="cuda"),
           torch.empty((k, 6), dtype=torch.int32, device="cuda"))
    ws = db.workspace(1, k)

    # ---- check this run's own output against the oracle on the returned entries ----
    import oracle
    db.query(qd, k, out=out, ws=ws)
    db.sync()
    idx = out[0].cpu().numpy()
    got_sc = out[1].cpu().numpy()
    _, o_cnt, o_sc = oracle.scan(gen, n, q, t_lo, t_hi, indices=idx.tolist())
    ok = bool(np.array_equal(o_sc.view(np.uint64), got_sc.view(np.uint64)) and
              np.array_equal(out[2].cpu().numpy().view(np.uint32).astype(np.uint64), o_cnt) and
              all(got_sc[i] >= got_sc[i + 1] for i in range(k - 1)))
    log(f"top-{k} re-checked by the oracle: {'ok' if ok else 'MISMATCH'}; source {src} "
        f"at rank {list(idx).index(src) if src in idx else '>k'}")

    # ---- timed region ----
    for _ in range(args.warmup):
        db.query(qd, k, out=out, ws=ws)
    torch.cuda.synchronize()
    db.profile(True)
    db.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        db.query(qd, k, out=out, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    scan_ms, launches = db.profile_read()
    db.profile(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    vox_per_s = n * V / ((t1 - t0) / args.steps)
    alg_bytes = n * 2 * (V // 8)
    scan_avg_ms = scan_ms / max(1, launches)
    achieved = alg_bytes / (scan_avg_ms * 1e-3) / 1e9
    traffic = load_traffic(args.workload)
    log(f"{ms_per_step:.3f} ms/query; scan kernel {scan_avg_ms:.3f} ms = {achieved:.0f} GB/s")

    cpu = None
    if args.cpu_seconds > 0:
        log("timing the CPU oracle sample")
        cpu = cpu_baseline(gen, q, t_lo, t_hi, args.cpu_seconds)
        log(f"cpu oracle {cpu['value']:.3e} voxels/s on {cpu['cores']} threads")

    latency = small_latency(db, qd, k, out, ws) if args.workload == "small" else None

    embed = None
    if args.workload == "full" and not args.no_embed:
        log("embedding search: held-out queries, fused latent search, exact rerank")
        embed = embed_run(args, db, gen, n, with_variants=False)

    line = {
        "metric": "database voxels compared/sec",
        "value": vox_per_s,
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"exact scan, {n} sims x {gen.nx}^3, bit-packed masks "
                               f"({alg_bytes / 1e9:.2f} GB), 1 query, top-{k}",
                   "n_db": n, "grid": [gen.nx, gen.ny, gen.nz], "k": k,
                   "thresholds": [t_lo, t_hi], "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "scan_kernel", "kernel_avg_ms": scan_avg_ms,
                     "algorithmic_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
        "parity": {"top_k_rechecked_by_oracle": ok},
        "build_s": build_s,
        "embed": embed,
    }
    if latency is not None:
        line["latency"] = latency
    print(json.dumps(line), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
