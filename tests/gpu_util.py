"""Helpers for GPU parity tests: device set-up, database builds, bit unpacking."""
import os
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(msg: str) -> None:
    print(msg, flush=True)


def unpack_planes(words: np.ndarray, nvox: int) -> np.ndarray:
    """uint32 words [..., Wp] (LSB-first) -> bool [..., nvox]."""
    w = np.ascontiguousarray(words).view(np.uint32)
    bits = np.unpackbits(w.view(np.uint8), axis=-1, bitorder="little")
    return bits[..., :nvox].astype(bool)


def build_db_from_host(gen: synth.GenConfig, n: int, t_lo: float, t_hi: float,
                       capacity: int | None = None, conc: np.ndarray | None = None,
                       chunk: int = 256):
    """Database from CPU-generated volumes (returns the db and the host volumes)."""
    from paper_2205_04550_amd import TumorDB
    if conc is None:
        conc = gen.conc_cpu(0, n)
    db = TumorDB(gen.nx, gen.ny, gen.nz, capacity or n, t_lo, t_hi)
    for s in range(0, n, chunk):
        db.append(torch.from_numpy(conc[s:s + chunk]).cuda())
    torch.cuda.synchronize()
    return db, conc


def build_db_on_gpu(gen: synth.GenConfig, n: int, t_lo: float, t_hi: float, chunk: int = 2048,
                    log=None):
    """Database from GPU-generated volumes, chunk by chunk (no host copy of the volumes)."""
    from paper_2205_04550_amd import TumorDB
    db = TumorDB(gen.nx, gen.ny, gen.nz, n, t_lo, t_hi)
    chunk = min(chunk, n)
    buf = torch.empty((chunk, gen.nvox), dtype=torch.float32, device="cuda")
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        p = torch.from_numpy(gen.params(s, c).view(np.float64).reshape(c, 8).copy()).cuda()
        gen.conc_gpu(p.data_ptr(), c, buf.data_ptr(), torch.cuda.current_stream().cuda_stream)
        db.append(buf[:c])
        if log and (s // chunk) % 8 == 0:
            log(f"  built {s + c}/{n}")
    torch.cuda.synchronize()
    del buf
    return db
