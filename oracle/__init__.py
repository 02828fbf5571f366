"""CPU oracle of the tumour-database retrieval scan.

TEST INFRASTRUCTURE ONLY: tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg use it; the GPU product path never does, and
this package imports nothing from it.

It is the paper's "Baseline for-loop search" (Sec. 2.3), written as the plain
definition: threshold every database volume into FLAIR and T1Gd masks
(Sec. 2.3), compute Dice against the query's two masks, add the two Dice
values, rank by the sum (highest wins). Per-voxel work is in ``oracle.c``;
ranking is a full sort here. Precision: counts are integers, Dice and the sum
are IEEE double.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> None:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-ffp-contract=off", os.path.join(HERE, "oracle.c"), "-o", _SO]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=HERE)


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.oracle_threshold.argtypes = [vp, i64, ctypes.c_float, ctypes.c_float, vp]
        lib.oracle_threshold.restype = None
        lib.oracle_counts.argtypes = [vp, vp, i32, i32, i32, vp, vp]
        lib.oracle_counts.restype = None
        lib.oracle_dice.argtypes = [ctypes.c_uint64] * 3
        lib.oracle_dice.restype = ctypes.c_double
        lib.oracle_score.argtypes = [vp]
        lib.oracle_score.restype = ctypes.c_double
        lib.oracle_scan_block.argtypes = [vp, i64, i32, i32, i32, ctypes.c_float, ctypes.c_float,
                                          vp, vp, vp, vp, i32]
        lib.oracle_scan_block.restype = None
        lib.oracle_scan_block_multi.argtypes = [vp, i64, i32, i32, i32, ctypes.c_float,
                                                ctypes.c_float, i32, vp, vp, vp, vp, i32]
        lib.oracle_scan_block_multi.restype = None
        _lib = lib
    return _lib


def host_cores() -> int:
    """Cores this process may run on (its CPU affinity set)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _threads() -> int:
    """Threads of the oracle's loops: every core of the affinity set, unless
    OMP_NUM_THREADS names fewer (a host that shares its cores between jobs sets it
    to this job's share)."""
    n = host_cores()
    env = os.environ.get("OMP_NUM_THREADS", "").strip()
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_model() -> str:
    """The host CPU's model name from /proc/cpuinfo ("unknown" if absent)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _roi_arg(roi):
    if roi is None:
        return None, None
    r = np.ascontiguousarray(np.asarray(roi, dtype=np.int32).reshape(6))
    return r, r.ctypes.data


def threshold(c: np.ndarray, t_lo: float, t_hi: float) -> np.ndarray:
    """Labels uint8, same shape: bit0 = c >= t_lo (FLAIR), bit1 = c >= t_hi (T1Gd)."""
    c = np.ascontiguousarray(c, dtype=np.float32)
    out = np.empty(c.shape, dtype=np.uint8)
    _L().oracle_threshold(c.ctypes.data, c.size, t_lo, t_hi, out.ctypes.data)
    return out


def counts(q: np.ndarray, lab: np.ndarray, roi=None) -> tuple:
    """(I_FL, I_T1, A_FL, A_T1, B_FL, B_T1) of query labels q vs labels lab [nz][ny][nx]."""
    q = np.ascontiguousarray(q, dtype=np.uint8)
    lab = np.ascontiguousarray(lab, dtype=np.uint8)
    assert q.shape == lab.shape and q.ndim == 3
    nz, ny, nx = q.shape
    out = np.zeros(6, dtype=np.uint64)
    r, rp = _roi_arg(roi)
    _L().oracle_counts(q.ctypes.data, lab.ctypes.data, nx, ny, nz, rp, out.ctypes.data)
    return tuple(int(v) for v in out)


def dice(I: int, A: int, B: int) -> float:
    return _L().oracle_dice(I, A, B)


def score(cnt) -> float:
    """Dice_T1Gd + Dice_FLAIR of one entry's counts."""
    a = np.ascontiguousarray(np.asarray(cnt, dtype=np.uint64).reshape(6))
    return _L().oracle_score(a.ctypes.data)


def scan_block(conc: np.ndarray, q: np.ndarray, t_lo: float, t_hi: float, roi=None,
               threads: int | None = None):
    """The for-loop over a block of volumes conc [n][nz][ny][nx] float32.

    Returns (counts uint64 [n][6], score float64 [n]).
    """
    conc = np.ascontiguousarray(conc, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.uint8)
    n = conc.shape[0]
    nz, ny, nx = conc.shape[1:]
    assert q.shape == (nz, ny, nx)
    cnt = np.zeros((n, 6), dtype=np.uint64)
    sc = np.zeros(n, dtype=np.float64)
    r, rp = _roi_arg(roi)
    if n:
        _L().oracle_scan_block(conc.ctypes.data, n, nx, ny, nz, t_lo, t_hi, q.ctypes.data, rp,
                               cnt.ctypes.data, sc.ctypes.data, threads or _threads())
    return cnt, sc


def scan_block_multi(conc: np.ndarray, queries: np.ndarray, t_lo: float, t_hi: float, rois=None,
                     threads: int | None = None):
    """scan_block for several queries at once (each entry thresholded once).

    queries: uint8 [nq][nz][ny][nx]; rois: int [nq][6] or None (whole grids).
    Returns (counts uint64 [nq][n][6], score float64 [nq][n]).
    """
    conc = np.ascontiguousarray(conc, dtype=np.float32)
    qs = np.ascontiguousarray(queries, dtype=np.uint8)
    n = conc.shape[0]
    nz, ny, nx = conc.shape[1:]
    nq = qs.shape[0]
    assert qs.shape[1:] == (nz, ny, nx)
    cnt = np.zeros((nq, n, 6), dtype=np.uint64)
    sc = np.zeros((nq, n), dtype=np.float64)
    rp = None
    if rois is not None:
        r = np.ascontiguousarray(np.asarray(rois, dtype=np.int32).reshape(nq, 6))
        rp = r.ctypes.data
    if n and nq:
        _L().oracle_scan_block_multi(conc.ctypes.data, n, nx, ny, nz, t_lo, t_hi, nq,
                                     qs.ctypes.data, rp, cnt.ctypes.data, sc.ctypes.data,
                                     threads or _threads())
    return cnt, sc


def rank(scores, k: int) -> list:
    """Indices of the k best entries: score descending, then index ascending (full sort)."""
    order = sorted(range(len(scores)), key=lambda n: (-float(scores[n]), n))
    return order[:k]


def scan(gen, n_db: int, q: np.ndarray, t_lo: float, t_hi: float, roi=None, chunk: int = 256,
         threads: int | None = None, indices=None):
    """Scores of database entries regenerated chunk by chunk from the generator config.

    ``gen`` is a ``synth.GenConfig``; ``indices`` (optional) restricts the loop
    to those entries. Returns (indices, counts [m][6], scores [m]).
    """
    idx = np.arange(n_db, dtype=np.int64) if indices is None else np.asarray(indices, np.int64)
    cnt = np.zeros((len(idx), 6), dtype=np.uint64)
    sc = np.zeros(len(idx), dtype=np.float64)
    if indices is None:
        for s in range(0, n_db, chunk):
            e = min(n_db, s + chunk)
            c, v = scan_block(gen.conc_cpu(s, e - s, threads), q, t_lo, t_hi, roi, threads)
            cnt[s:e], sc[s:e] = c, v
    else:
        for j, n in enumerate(idx):
            c, v = scan_block(gen.conc_cpu(int(n), 1, threads), q, t_lo, t_hi, roi, threads)
            cnt[j], sc[j] = c[0], v[0]
    return idx, cnt, sc


def query(gen, n_db: int, q: np.ndarray, k: int, t_lo: float, t_hi: float, roi=None,
          chunk: int = 256, threads: int | None = None):
    """Top-k of the exhaustive loop: (idx [k], score [k], counts [k][6])."""
    _, cnt, sc = scan(gen, n_db, q, t_lo, t_hi, roi, chunk, threads)
    top = rank(sc, k)
    return np.array(top, dtype=np.int64), sc[top], cnt[top]


def resample_nearest(labels: np.ndarray, shape) -> np.ndarray:
    """Order-0 spline (nearest-neighbour) resampling of label volumes [..., nz, ny, nx] to
    [..., *shape] with scipy.ndimage.zoom, the routine the paper used for DS64 / DS32
    (Sec. 2.3); a library primitive used as one step."""
    import scipy.ndimage as nd
    lab = np.asarray(labels)
    lead = lab.ndim - 3
    factors = [1.0] * lead + [o / i for o, i in zip(shape, lab.shape[lead:])]
    out = nd.zoom(lab, factors, order=0)
    assert out.shape[lead:] == tuple(shape), (out.shape, shape)
    return out


def moments(labels: np.ndarray) -> tuple:
    """(sum x, sum y, sum z, count) over the FLAIR voxels (bit0) of labels [nz][ny][nx].

    Their ratios are the tumour's centre of mass, the location feature of the
    paper's radiomics query (Sec. 2.3)."""
    z, y, x = np.nonzero(np.asarray(labels) & 1)
    return int(x.sum()), int(y.sum()), int(z.sum()), int(x.size)


def rowbox(labels: np.ndarray) -> tuple:
    """(z0, z1, y0, y1): half-open range of the x-rows holding any FLAIR or T1Gd voxel;
    (0, 0, 0, 0) when there is none."""
    rows = np.any((np.asarray(labels) & 3) != 0, axis=2)   # [nz][ny]
    z, y = np.nonzero(rows)
    if z.size == 0:
        return 0, 0, 0, 0
    return int(z.min()), int(z.max()) + 1, int(y.min()), int(y.max()) + 1


def com_key(qm: tuple, em: tuple) -> np.float32:
    """Squared distance of two centres of mass from their moments, in double (centre =
    sum / count; squares added x, y, z), rounded once to float32; +inf if either mask is
    empty."""
    if qm[3] == 0 or em[3] == 0:
        return np.float32(np.inf)
    d = [float(qm[i]) / float(qm[3]) - float(em[i]) / float(em[3]) for i in range(3)]
    return np.float32(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])


def query_com(q: np.ndarray, labs: np.ndarray, n_cand: int, k: int):
    """Centre-of-mass prefilter then exact Dice on the candidates (Sec. 2.3 radiomics
    query's location step; candidates re-scored by the baseline score).

    q: labels [nz][ny][nx]; labs: database labels [n][nz][ny][nx]. Returns
    (cand [n_cand], cand_key float32 [n_cand], top [k], score [k], counts [k][6])."""
    qm = moments(q)
    keys = np.array([com_key(qm, moments(l)) for l in labs], dtype=np.float32)
    cand = sorted(range(len(labs)), key=lambda n: (float(keys[n]), n))[:n_cand]
    cnt = np.array([counts(q, labs[n]) for n in cand], dtype=np.uint64)
    sc = np.array([score(c) for c in cnt])
    order = rank(sc, k)
    return (np.array(cand), keys[cand], np.array([cand[j] for j in order]), sc[order],
            cnt[order])
