"""Seeded synthetic inputs for the tumour-database retrieval scan.

The paper's database (50,000 reaction-diffusion simulations on 128^3 in the
SRI24 atlas, Sec. 3 "Data") and its 62 patient segmentations are not
available. This module manufactures stand-ins with the same shapes: logistic
tumour fronts inside an ellipsoidal brain mask, and noisy two-mask patient
segmentations. It holds none of the retrieval method's arithmetic and is the
only code shared by the oracle side and the GPU side (both read its bytes).

CPU generation is ``libsynth.so`` (gcc, OpenMP); GPU generation of the same
bytes is ``libsynth_gpu.so`` (hipcc). Both evaluate ``synth_formula.h``.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_CPU_SO = os.path.join(HERE, "libsynth.so")
_GPU_SO = os.path.join(HERE, "libsynth_gpu.so")

PARAM_DTYPE = np.dtype([(n, np.float64) for n in ("cx", "cy", "cz", "iax", "iay", "iaz", "R", "iw")])

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
             "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> None:
    """Compile the CPU and GPU generators in place."""
    cmds = [
        ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
         "-fno-fast-math", os.path.join(HERE, "synth_cpu.c"), "-o", _CPU_SO, "-lm"],
        ["hipcc", *HIP_FLAGS, os.path.join(HERE, "synth_gpu.hip"), "-o", _GPU_SO],
    ]
    for c in cmds:
        if verbose:
            print(" ".join(c), flush=True)
        subprocess.run(c, check=True, cwd=HERE)


_cpu = None
_gpu = None


def _cpu_lib():
    global _cpu
    if _cpu is None:
        if not os.path.exists(_CPU_SO):
            build()
        lib = ctypes.CDLL(_CPU_SO)
        lib.synth_uniform.restype = ctypes.c_double
        lib.synth_uniform.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint64]
        lib.synth_params.restype = None
        lib.synth_params.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        lib.synth_fill_cpu.restype = None
        lib.synth_fill_cpu.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
        lib.synth_query_labels.restype = ctypes.c_int
        lib.synth_query_labels.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_float, ctypes.c_float, ctypes.c_uint64,
                                           ctypes.c_int64, ctypes.c_double, ctypes.c_void_p,
                                           ctypes.c_void_p]
        _cpu = lib
    return _cpu


def _gpu_lib():
    global _gpu
    if _gpu is None:
        if not os.path.exists(_GPU_SO):
            raise RuntimeError(f"{_GPU_SO} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(_GPU_SO)
        lib.synth_fill_gpu.restype = ctypes.c_int
        lib.synth_fill_gpu.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        _gpu = lib
    return _gpu


def uniform(seed: int, item: int, draw: int) -> float:
    return _cpu_lib().synth_uniform(seed, item, draw)


def default_threads() -> int:
    """Every core of the affinity set, unless OMP_NUM_THREADS names fewer."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "").strip()
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


@dataclasses.dataclass(frozen=True)
class GenConfig:
    """One synthetic database: grid, radius/width ranges, seed."""
    nx: int
    ny: int
    nz: int
    r_lo: float
    r_hi: float
    w_lo: float
    w_hi: float
    seed: int

    @property
    def nvox(self) -> int:
        return self.nx * self.ny * self.nz

    def params(self, n0: int, count: int, seed: int | None = None) -> np.ndarray:
        out = np.zeros(count, dtype=PARAM_DTYPE)
        if count:
            _cpu_lib().synth_params(self.seed if seed is None else seed, n0, count, self.nx,
                                    self.ny, self.nz, self.r_lo, self.r_hi, self.w_lo, self.w_hi,
                                    out.ctypes.data)
        return out

    def conc_cpu(self, n0: int, count: int, threads: int | None = None,
                 seed: int | None = None) -> np.ndarray:
        """float32 [count][nz][ny][nx] on the host."""
        p = self.params(n0, count, seed)
        out = np.empty((count, self.nz, self.ny, self.nx), dtype=np.float32)
        if count:
            _cpu_lib().synth_fill_cpu(p.ctypes.data, count, self.nx, self.ny, self.nz,
                                      out.ctypes.data, threads or default_threads())
        return out

    def conc_gpu(self, params_dev_ptr: int, count: int, out_ptr: int, stream: int = 0) -> None:
        """Fill float32 [count][V] at out_ptr from a device parameter table."""
        rc = _gpu_lib().synth_fill_gpu(params_dev_ptr, count, self.nx, self.ny, self.nz,
                                       out_ptr, stream)
        if rc != 0:
            raise RuntimeError(f"synth_fill_gpu failed ({rc})")

    def query(self, src: int, t_lo: float, t_hi: float, noise_seed: int, qid: int,
              flip_frac: float = 0.02, seed: int | None = None) -> np.ndarray:
        """uint8 [nz][ny][nx] patient stand-in: bit0 FLAIR, bit1 T1Gd."""
        p = self.params(src, 1, seed)
        lab = np.empty((self.nz, self.ny, self.nx), dtype=np.uint8)
        nflip = np.zeros(2, dtype=np.int64)
        rc = _cpu_lib().synth_query_labels(p.ctypes.data, self.nx, self.ny, self.nz, t_lo, t_hi,
                                           noise_seed, qid, flip_frac, lab.ctypes.data,
                                           nflip.ctypes.data)
        if rc != 0:
            raise MemoryError("synth_query_labels")
        return lab


# Workloads (sizes and distributions of the paper's database, Sec. 3).
T_LO, T_HI = 0.25, 0.675     # FLAIR / T1Gd segmentation thresholds of the workloads
PAPER_T_LO, PAPER_T_HI = 0.2, 0.6  # the paper's own values (Sec. 2.3)
DB_SEED, QUERY_SEED, BATCH_QUERY_SEED, ROI_SEED, HELDOUT_SEED = 2205, 4550, 4551, 4552, 4553

SMALL = GenConfig(64, 64, 64, 4.0, 20.0, 0.5, 4.0, DB_SEED)     # 1,000 sims, 64^3
FULL = GenConfig(128, 128, 128, 8.0, 40.0, 1.0, 8.0, DB_SEED)   # 50,000 sims, 128^3
SMALL_N, FULL_N = 1000, 50000


def query_source(n_db: int, query_seed: int, qid: int) -> int:
    """Database entry a noisy self-query is made from."""
    return min(n_db - 1, int(math.floor(uniform(query_seed, qid, 0) * n_db)))


def make_queries(cfg: GenConfig, n_db: int, nq: int, query_seed: int, t_lo: float = T_LO,
                 t_hi: float = T_HI, flip_frac: float = 0.02, held_out_seed: int | None = None):
    """nq noisy queries [nq][nz][ny][nx] uint8 and their source indices.

    With held_out_seed the sources are simulations of that seed (not in the
    database), as the paper's 1k held-out synthetic evaluation set (Sec. 3).
    """
    labs = np.empty((nq, cfg.nz, cfg.ny, cfg.nx), dtype=np.uint8)
    srcs = np.empty(nq, dtype=np.int64)

    def one(q):
        if held_out_seed is None:
            s = query_source(n_db, query_seed, q)
            labs[q] = cfg.query(s, t_lo, t_hi, query_seed, q, flip_frac)
        else:
            s = q
            labs[q] = cfg.query(s, t_lo, t_hi, query_seed, q, flip_frac, seed=held_out_seed)
        srcs[q] = s

    # Each query is independent and the C generator releases the GIL.
    if nq > 4:
        import concurrent.futures as cf
        with cf.ThreadPoolExecutor(max_workers=default_threads()) as ex:
            list(ex.map(one, range(nq)))
    else:
        for q in range(nq):
            one(q)
    return labs, srcs


def make_rois(labels: np.ndarray, roi_seed: int, side_lo: int = 24, side_hi: int = 128) -> np.ndarray:
    """Per-query half-open boxes int32 [nq][6] = (x0, y0, z0, x1, y1, z1).

    Side per axis ~ U{side_lo .. min(side_hi, n_d)}, centred on the query's
    FLAIR bounding-box centre (grid centre when empty) and shifted inside the
    grid. The box may crop the tumour.
    """
    nq, nz, ny, nx = labels.shape
    dims = (nx, ny, nz)
    out = np.zeros((nq, 6), dtype=np.int32)
    for q in range(nq):
        fl = (labels[q] & 1) != 0
        if fl.any():
            zs, ys, xs = np.nonzero(fl)
            ctr = ((xs.min() + xs.max() + 1) / 2.0, (ys.min() + ys.max() + 1) / 2.0,
                   (zs.min() + zs.max() + 1) / 2.0)
        else:
            ctr = (nx / 2.0, ny / 2.0, nz / 2.0)
        for d in range(3):
            hi = min(side_hi, dims[d])
            lo_s = min(side_lo, hi)
            s = lo_s + min(hi - lo_s, int(math.floor(uniform(roi_seed, q, d) * (hi - lo_s + 1))))
            lo = int(math.floor(ctr[d] - s / 2.0 + 0.5))
            lo = max(0, min(dims[d] - s, lo))
            out[q, d] = lo
            out[q, d + 3] = lo + s
    return out
