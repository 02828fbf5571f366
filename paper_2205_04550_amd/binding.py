"""ctypes binding of libtumordb (include/tumordb.h) with torch for device memory and streams.

Argument marshalling only: every step of the retrieval runs in the HIP
kernels of libtumordb.so. There is no fallback: if the library is missing
the import fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtumordb.so")

DB_OK, DB_EINVAL, DB_ENOMEM, DB_EHIP, DB_ESTATE, DB_ENOSPC = 0, -1, -2, -3, -4, -5
DB_KMAX = 1024
SYMBOLS = ("db_storage_bytes", "db_build", "db_append", "db_size", "db_query_workspace_bytes",
           "db_scan", "db_query", "db_query_batch", "db_sync", "db_free", "db_last_error",
           "db_profile", "db_profile_read", "emb_quantize", "emb_distances", "emb_topk_min",
           "emb_topk_min_workspace_bytes",
           "db_rerank_workspace_bytes", "db_rerank", "db_query_embed_workspace_bytes",
           "db_query_embed", "db_tune_batch", "db_append_resampled", "labels_resample",
           "db_query_sparse", "db_query_com_workspace_bytes", "db_query_com",
           "emb_hash_thresholds", "emb_binarize", "emb_distances_l2sum", "db_rerank_pack",
           "db_rerank_packed", "emb_groups_workspace_bytes", "emb_distances_groups",
           "emb_topk_groups", "db_query_noalloc", "emb_knn_workspace_bytes", "emb_knn",
           "db_rerank_pack_pool", "db_set_rerank_bound")
EMB_BF16, EMB_FP8, EMB_BIN = 0, 1, 2


class DbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class RoiT(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("x0", "y0", "z0", "x1", "y1", "z1")]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(python -m paper_2205_04550_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "db_storage_bytes": (sz, [i32, i32, i32, i64]),
        "db_build": (i32, [ctypes.POINTER(vp), i32, i32, i32, ctypes.c_float, ctypes.c_float,
                           i64, vp, sz]),
        "db_append": (i32, [vp, vp, i64, vp]),
        "db_size": (i64, [vp]),
        "db_query_workspace_bytes": (sz, [vp, i32, i32]),
        "db_scan": (i32, [vp, vp, vp, vp, vp, sz, vp]),
        "db_query": (i32, [vp, vp, i32, vp, vp, vp, vp, sz, vp]),
        "db_query_noalloc": (i32, [vp, vp, i32, vp, vp, vp, vp]),
        "db_query_batch": (i32, [vp, i32, vp, vp, i32, vp, vp, vp, vp, sz, vp]),
        "db_query_sparse": (i32, [vp, vp, i32, vp, vp, vp, vp, sz, vp]),
        "db_query_com_workspace_bytes": (sz, [vp, i32, i32]),
        "db_query_com": (i32, [vp, i32, vp, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp]),
        "db_sync": (i32, [vp, vp]),
        "db_free": (None, [vp]),
        "db_last_error": (ctypes.c_char_p, []),
        "db_profile": (i32, [vp, i32]),
        "db_tune_batch": (i32, [vp, i32, i32, i32, i32]),
        "db_set_rerank_bound": (i32, [vp, i32]),
        "db_append_resampled": (i32, [vp, vp, i64, i64, vp]),
        "labels_resample": (i32, [i32, vp, i32, i32, i32, vp, i32, i32, i32, vp]),
        "emb_quantize": (i32, [i64, i32, vp, i32, vp, vp, vp, vp]),
        "emb_distances": (i32, [i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]),
        "emb_topk_min": (i32, [i32, i32, vp, i32, vp, vp, vp, sz, vp]),
        "emb_topk_min_workspace_bytes": (sz, [i32, i32, i32]),
        "emb_groups_workspace_bytes": (sz, [i32, i32]),
        "emb_distances_groups": (i32, [i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
        "emb_topk_groups": (i32, [i32, i32, vp, i32, vp, vp, vp, sz, vp]),
        "emb_knn_workspace_bytes": (sz, [i32, i32, i32]),
        "emb_knn": (i32, [i32, i32, i32, i32] + [vp] * 6 + [i32, i32, vp, vp, vp, sz, vp]),
        "emb_hash_thresholds": (i32, [i64, i32, vp, vp, vp]),
        "emb_distances_l2sum": (i32, [i32, i32, i32, i32] + [vp] * 12 + [vp, vp]),
        "emb_binarize": (i32, [i64, i32, vp, vp, vp, vp]),
        "db_rerank_workspace_bytes": (sz, [vp, i32]),
        "db_rerank": (i32, [vp, i32, vp, vp, i32, i32, vp, vp, vp, vp, sz, vp]),
        "db_rerank_pack": (i32, [vp, i32, vp, vp, sz, vp]),
        "db_rerank_pack_pool": (i32, [vp, i32, vp, vp, vp, sz, vp]),
        "db_rerank_packed": (i32, [vp, i32, vp, i32, i32, vp, vp, vp, vp, sz, vp]),
        "db_query_embed_workspace_bytes": (sz, [vp, i32, i32]),
        "db_query_embed": (i32, [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, i32, i32, vp, vp,
                                 vp, vp, vp, vp, sz, vp]),
        "db_profile_read": (i32, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def _check(rc: int) -> None:
    if rc != DB_OK:
        raise DbError(rc, LIB.db_last_error().decode())


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def storage_bytes(nx: int, ny: int, nz: int, capacity: int) -> int:
    return LIB.db_storage_bytes(nx, ny, nz, capacity)


class TumorDB:
    """A database of bit-packed FLAIR/T1Gd masks resident in device memory."""

    def __init__(self, nx: int, ny: int, nz: int, capacity: int, t_lo: float, t_hi: float,
                 device: str | torch.device = "cuda"):
        nbytes = storage_bytes(nx, ny, nz, capacity)
        if nbytes == 0:
            raise DbError(DB_EINVAL, f"bad grid {nx}x{ny}x{nz} or capacity {capacity}")
        self.dims = (nx, ny, nz)
        self.capacity = capacity
        self.t_lo, self.t_hi = t_lo, t_hi
        self.storage = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(LIB.db_build(ctypes.byref(h), nx, ny, nz, t_lo, t_hi, capacity,
                            self.storage.data_ptr(), nbytes))
        self._h = h
        self.W = nx * ny * nz // 32
        self.Wp = (self.W + 3) // 4 * 4
        self._ws = {}

    # ---- build --------------------------------------------------------------------------
    def append(self, conc: torch.Tensor, stream=None) -> None:
        """Threshold + pack float32 densities [n][nz][ny][nx] (device)."""
        nx, ny, nz = self.dims
        assert conc.dtype == torch.float32 and conc.is_cuda and conc.is_contiguous()
        assert conc.numel() % (nx * ny * nz) == 0
        n = conc.numel() // (nx * ny * nz)
        _check(LIB.db_append(self._h, conc.data_ptr(), n, _stream(stream)))

    def __len__(self) -> int:
        return LIB.db_size(self._h)

    @property
    def planes(self) -> torch.Tensor:
        """int32 view [capacity][2][Wp] of the packed masks (bits are uint32 words)."""
        nb = self.capacity * 2 * self.Wp * 4
        return self.storage[:nb].view(torch.int32).view(self.capacity, 2, self.Wp)

    def _offsets(self):
        up = lambda b: (b + 255) // 256 * 256
        pc = up(self.capacity * 2 * self.Wp * 4)
        box = pc + up(self.capacity * 8)
        mom = box + up(self.capacity * 16)
        order = mom + up(self.capacity * 32)
        tbox = order + up(self.capacity * 4)
        zrange = tbox + up(self.capacity * 16)
        bcnt = zrange + up(self.capacity * self.dims[2] * 8)
        return pc, box, mom, order, tbox, zrange, bcnt

    def block_dims(self):
        """(nbx, nby, nbz, nbp) of the per-entry 16^3-block counts (nbp = 0: none kept)."""
        nx, ny, nz = self.dims
        nbx, nby, nbz = nx // 16, (ny + 15) // 16, (nz + 15) // 16
        nb = nbx * nby * nbz
        return nbx, nby, nbz, ((nb + 7) // 8 * 8 if nb <= 2048 else 0)

    @property
    def popcounts(self) -> torch.Tensor:
        """int32 view [capacity][2] of |B_FLAIR|, |B_T1Gd|."""
        off = self._offsets()[0]
        return self.storage[off:off + self.capacity * 8].view(torch.int32).view(self.capacity, 2)

    @property
    def boxes(self) -> torch.Tensor:
        """int32 view [capacity][4] of the row boxes z0, z1, y0, y1 of the set bits."""
        off = self._offsets()[1]
        return self.storage[off:off + self.capacity * 16].view(torch.int32).view(self.capacity, 4)

    @property
    def tboxes(self) -> torch.Tensor:
        """int32 view [capacity][4] of the row boxes z0, z1, y0, y1 of the T1Gd bits alone."""
        off = self._offsets()[4]
        return self.storage[off:off + self.capacity * 16].view(torch.int32).view(self.capacity, 4)

    @property
    def zranges(self) -> torch.Tensor:
        """int32 view [capacity][nz][2] of the per z-slice y-ranges of the FLAIR and the T1Gd
        rows, each y0 | y1 << 16 ([y0, y1); 0 for a slice without such rows)."""
        off = self._offsets()[5]
        return (self.storage[off:off + self.capacity * self.dims[2] * 8].view(torch.int32)
                .view(self.capacity, self.dims[2], 2))

    @property
    def block_counts(self) -> torch.Tensor:
        """int16 view [capacity][2][nbp] of the set voxels per 16^3 block and mask (uint16
        values; block (bz, by, bx) at (bz nby + by) nbx + bx)."""
        nbp = self.block_dims()[3]
        off = self._offsets()[6]
        return (self.storage[off:off + self.capacity * 4 * nbp].view(torch.int16)
                .view(self.capacity, 2, nbp))

    @property
    def tile_order(self) -> torch.Tensor:
        """int32 view [capacity] of the entry order of the batched scan's tiles (valid after a
        batched query)."""
        off = self._offsets()[3]
        return self.storage[off:off + self.capacity * 4].view(torch.int32)

    @property
    def moments(self) -> torch.Tensor:
        """int64 view [capacity][4] of the FLAIR moments (sum x, sum y, sum z, count)."""
        off = self._offsets()[2]
        return self.storage[off:off + self.capacity * 32].view(torch.int64).view(self.capacity, 4)

    # ---- query --------------------------------------------------------------------------
    def workspace_bytes(self, nq: int, k: int) -> int:
        return LIB.db_query_workspace_bytes(self._h, nq, k)

    def workspace(self, nq: int, k: int) -> torch.Tensor:
        nb = self.workspace_bytes(nq, k)
        if nb == 0:
            raise DbError(DB_EINVAL, f"bad workspace request nq={nq} k={k}")
        ws = self._ws.get((nq, k))
        if ws is None or ws.numel() < nb:
            ws = torch.empty(nb, dtype=torch.uint8, device=self.storage.device)
            self._ws[(nq, k)] = ws
        return ws

    def scan(self, q_labels: torch.Tensor, inter: torch.Tensor | None = None,
             qcount: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None):
        """Intersections [N][2] (int32 holding uint32) and query counts [2]."""
        n = len(self)
        dev = self.storage.device
        inter = torch.empty((n, 2), dtype=torch.int32, device=dev) if inter is None else inter
        qcount = torch.empty(2, dtype=torch.int32, device=dev) if qcount is None else qcount
        ws = self.workspace(1, 1) if ws is None else ws
        _check(LIB.db_scan(self._h, q_labels.data_ptr(), inter.data_ptr(), qcount.data_ptr(),
                           ws.data_ptr(), ws.numel(), _stream(stream)))
        return inter, qcount

    def query(self, q_labels: torch.Tensor, k: int, with_counts: bool = True, out=None,
              ws: torch.Tensor | None = None, stream=None):
        """Top-k (idx int32 [k], score float64 [k], counts int32 [k][6] or None)."""
        dev = self.storage.device
        if out is None:
            idx = torch.empty(k, dtype=torch.int32, device=dev)
            score = torch.empty(k, dtype=torch.float64, device=dev)
            counts = torch.empty((k, 6), dtype=torch.int32, device=dev) if with_counts else None
        else:
            idx, score, counts = out
        ws = self.workspace(1, k) if ws is None else ws
        _check(LIB.db_query(self._h, q_labels.data_ptr(), k, idx.data_ptr(), score.data_ptr(),
                            _ptr(counts), ws.data_ptr(), ws.numel(), _stream(stream)))
        return idx, score, counts

    def query_noalloc(self, q_labels: torch.Tensor, k: int, with_counts: bool = True, out=None,
                      stream=None):
        """query() with the library's fixed device scratch array instead of a workspace
        (db_query_noalloc: nothing is allocated by the call; outputs are allocated here
        unless given in out)."""
        dev = self.storage.device
        if out is None:
            idx = torch.empty(k, dtype=torch.int32, device=dev)
            score = torch.empty(k, dtype=torch.float64, device=dev)
            counts = torch.empty((k, 6), dtype=torch.int32, device=dev) if with_counts else None
        else:
            idx, score, counts = out
        _check(LIB.db_query_noalloc(self._h, q_labels.data_ptr(), k, idx.data_ptr(),
                                    score.data_ptr(), _ptr(counts), _stream(stream)))
        return idx, score, counts

    def query_sparse(self, q_labels: torch.Tensor, k: int, with_counts: bool = True, out=None,
                     ws: torch.Tensor | None = None, stream=None):
        """query() computed over the rows inside both boxes only (same results)."""
        dev = self.storage.device
        if out is None:
            idx = torch.empty(k, dtype=torch.int32, device=dev)
            score = torch.empty(k, dtype=torch.float64, device=dev)
            counts = torch.empty((k, 6), dtype=torch.int32, device=dev) if with_counts else None
        else:
            idx, score, counts = out
        ws = self.workspace(1, k) if ws is None else ws
        _check(LIB.db_query_sparse(self._h, q_labels.data_ptr(), k, idx.data_ptr(),
                                   score.data_ptr(), _ptr(counts), ws.data_ptr(), ws.numel(),
                                   _stream(stream)))
        return idx, score, counts

    def query_com(self, q_labels: torch.Tensor, n_cand: int, k: int, ws: torch.Tensor | None = None,
                  out=None, stream=None):
        """Centre-of-mass prefilter (n_cand nearest) + exact rerank ->
        (idx, score, counts, cand_idx, cand_d)."""
        nq = q_labels.shape[0]
        dev = self.storage.device
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int32, device=dev),
                   torch.empty((nq, k), dtype=torch.float64, device=dev),
                   torch.empty((nq, k, 6), dtype=torch.int32, device=dev),
                   torch.empty((nq, n_cand), dtype=torch.int32, device=dev),
                   torch.empty((nq, n_cand), dtype=torch.float32, device=dev))
        if ws is None:
            ws = torch.empty(LIB.db_query_com_workspace_bytes(self._h, nq, n_cand),
                             dtype=torch.uint8, device=dev)
        idx, score, counts, ci, cd = out
        _check(LIB.db_query_com(self._h, nq, q_labels.data_ptr(), n_cand, k, idx.data_ptr(),
                                score.data_ptr(), _ptr(counts), _ptr(ci), _ptr(cd), ws.data_ptr(),
                                ws.numel(), _stream(stream)))
        return out

    def query_batch(self, q_labels: torch.Tensor, rois, k: int, with_counts: bool = True,
                    out=None, ws: torch.Tensor | None = None, stream=None):
        """nq queries [nq][nz][ny][nx] with boxes int [nq][6] (x0,y0,z0,x1,y1,z1) or None."""
        nq = q_labels.shape[0]
        dev = self.storage.device
        if out is None:
            idx = torch.empty((nq, k), dtype=torch.int32, device=dev)
            score = torch.empty((nq, k), dtype=torch.float64, device=dev)
            counts = torch.empty((nq, k, 6), dtype=torch.int32, device=dev) if with_counts else None
        else:
            idx, score, counts = out
        roi_arr = None
        rp = None
        if rois is not None:
            roi_arr = np.ascontiguousarray(np.asarray(rois, dtype=np.int32).reshape(nq, 6))
            rp = roi_arr.ctypes.data
        ws = self.workspace(nq, k) if ws is None else ws
        _check(LIB.db_query_batch(self._h, nq, q_labels.data_ptr(), rp, k, idx.data_ptr(),
                                  score.data_ptr(), _ptr(counts), ws.data_ptr(), ws.numel(),
                                  _stream(stream)))
        return idx, score, counts

    def rerank(self, q_labels: torch.Tensor, cand: torch.Tensor, k: int, stream=None):
        """Exact Dice re-scoring of candidate entries cand [nq][nc] (int32): top-k per query."""
        nq, nc = cand.shape
        dev = self.storage.device
        idx = torch.empty((nq, k), dtype=torch.int32, device=dev)
        score = torch.empty((nq, k), dtype=torch.float64, device=dev)
        counts = torch.empty((nq, k, 6), dtype=torch.int32, device=dev)
        nb = LIB.db_rerank_workspace_bytes(self._h, nq)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        cand = cand.to(torch.int32).contiguous()
        _check(LIB.db_rerank(self._h, nq, q_labels.data_ptr(), cand.data_ptr(), nc, k,
                             idx.data_ptr(), score.data_ptr(), counts.data_ptr(), ws.data_ptr(), nb,
                             _stream(stream)))
        return idx, score, counts

    def rerank_workspace(self, nq: int) -> torch.Tensor:
        """A workspace for rerank / rerank_pack + rerank_packed of nq queries."""
        nb = LIB.db_rerank_workspace_bytes(self._h, nq)
        return torch.empty(nb, dtype=torch.uint8, device=self.storage.device)

    def rerank_pack(self, q_labels: torch.Tensor, ws: torch.Tensor, stream=None) -> None:
        """First half of rerank: pack the queries q_labels [nq][nz][ny][nx] into ws."""
        _check(LIB.db_rerank_pack(self._h, q_labels.shape[0], q_labels.data_ptr(), ws.data_ptr(),
                                  ws.numel(), _stream(stream)))

    def rerank_pack_pool(self, q_labels: torch.Tensor, ws: torch.Tensor,
                         pooled: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """rerank_pack that also returns the labels' pooled counts, uint8 [nq][nz/2][ny/2][nx/2]
        (per 2x2x2 block: FLAIR count in bits 0..3, T1Gd count in bits 4..7), the input of
        the encoder's first layer from the same read of the labels."""
        nq, nz, ny, nx = q_labels.shape
        shape = (nq, nz // 2, ny // 2, nx // 2)
        if pooled is None:
            pooled = torch.empty(shape, dtype=torch.uint8, device=q_labels.device)
        assert pooled.dtype == torch.uint8 and tuple(pooled.shape) == shape and pooled.is_contiguous()
        _check(LIB.db_rerank_pack_pool(self._h, nq, q_labels.data_ptr(), pooled.data_ptr(),
                                       ws.data_ptr(), ws.numel(), _stream(stream)))
        return pooled

    def packed_queries(self, ws: torch.Tensor, nq: int) -> torch.Tensor:
        """int32 view [nq][2][Wp] of the queries' packed masks that rerank_pack left at the start
        of ws (the database's plane layout)."""
        return ws[:nq * 2 * self.Wp * 4].view(torch.int32).view(nq, 2, self.Wp)

    def rerank_packed(self, ws: torch.Tensor, cand: torch.Tensor, k: int, stream=None):
        """Second half of rerank: score cand [nq][nc] against the queries packed into ws."""
        nq, nc = cand.shape
        dev = self.storage.device
        idx = torch.empty((nq, k), dtype=torch.int32, device=dev)
        score = torch.empty((nq, k), dtype=torch.float64, device=dev)
        counts = torch.empty((nq, k, 6), dtype=torch.int32, device=dev)
        cand = cand.to(torch.int32).contiguous()
        _check(LIB.db_rerank_packed(self._h, nq, cand.data_ptr(), nc, k, idx.data_ptr(),
                                    score.data_ptr(), counts.data_ptr(), ws.data_ptr(), ws.numel(),
                                    _stream(stream)))
        return idx, score, counts

    def query_embed(self, fmt: int, q: "Latents", x: "Latents", q_labels: torch.Tensor,
                    n_cand: int, k: int, ws: torch.Tensor | None = None, out=None, stream=None):
        """Latent search (n_cand nearest) + exact rerank -> (idx, score, counts, cand_idx, cand_d)."""
        nq = q.codes.shape[0]
        dev = self.storage.device
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int32, device=dev),
                   torch.empty((nq, k), dtype=torch.float64, device=dev),
                   torch.empty((nq, k, 6), dtype=torch.int32, device=dev),
                   torch.empty((nq, n_cand), dtype=torch.int32, device=dev),
                   torch.empty((nq, n_cand), dtype=torch.float32, device=dev))
        if ws is None:
            ws = torch.empty(LIB.db_query_embed_workspace_bytes(self._h, nq, n_cand),
                             dtype=torch.uint8, device=dev)
        idx, score, counts, ci, cd = out
        _check(LIB.db_query_embed(self._h, fmt, nq, q.dim, q.codes.data_ptr(), _ptr(q.scale),
                                  _ptr(q.sq), x.codes.data_ptr(), _ptr(x.scale), _ptr(x.sq),
                                  q_labels.data_ptr(), n_cand, k, idx.data_ptr(), score.data_ptr(),
                                  counts.data_ptr(), ci.data_ptr(), cd.data_ptr(), ws.data_ptr(),
                                  ws.numel(), _stream(stream)))
        return out

    def append_resampled(self, src: "TumorDB", first: int = 0, n: int | None = None,
                         stream=None) -> None:
        """Append src's entries resampled (order 0) to this database's grid."""
        n = len(src) - first if n is None else n
        _check(LIB.db_append_resampled(self._h, src._h, first, n, _stream(stream)))

    def tune_batch(self, slab_planes: int = 0, block_threads: int = 0, tile_entries: int = 0,
                   query_chunk: int = 0) -> None:
        """Launch shape of query_batch (0 = defaults; slab_planes = -1 selects the kernel that
        reads the database through L2); results are the same for any shape."""
        _check(LIB.db_tune_batch(self._h, slab_planes, block_threads, tile_entries, query_chunk))

    def set_rerank_bound(self, on: bool) -> None:
        """Rerank in bound order, leaving out candidates that cannot reach the top k (the
        default), or score every candidate; results are the same either way."""
        _check(LIB.db_set_rerank_bound(self._h, 1 if on else 0))

    def profile(self, enable: bool) -> None:
        """Record HIP events around the dominant kernel of every later query call."""
        _check(LIB.db_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """(summed milliseconds, launches) of the dominant kernel since the last read."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(LIB.db_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def sync(self, stream=None) -> None:
        _check(LIB.db_sync(self._h, _stream(stream)))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            LIB.db_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _hand_to(stream, *tensors) -> None:
    """Use on `stream` of tensors made on the current stream: the stream waits for the
    current stream's work so far (the tensors' contents), and the caching allocator keeps
    their memory until the stream's work on them is done (record_stream)."""
    if stream is None or stream == torch.cuda.current_stream(stream.device):
        return
    stream.wait_stream(torch.cuda.current_stream(stream.device))
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


class Latents:
    """Quantised latents on the device: codes [n][dim] (bf16 bits or e4m3 bytes), per-row
    scale (FP8 only) and squared norm of the stored vectors."""

    def __init__(self, lat: torch.Tensor, fmt: int, stream=None):
        lat = lat.to(torch.float32).contiguous()
        n, dim = lat.shape
        self.fmt, self.n, self.dim = fmt, n, dim
        dev = lat.device
        if fmt == EMB_BF16:
            self.codes = torch.empty((n, dim), dtype=torch.bfloat16, device=dev)
            self.scale = None
        else:
            self.codes = torch.empty((n, dim), dtype=torch.uint8, device=dev)
            self.scale = torch.empty(n, dtype=torch.float32, device=dev)
        self.sq = torch.empty(n, dtype=torch.float32, device=dev)
        _hand_to(stream, lat, self.codes, self.scale, self.sq)
        _check(LIB.emb_quantize(n, dim, lat.data_ptr(), fmt, self.codes.data_ptr(), _ptr(self.scale),
                                self.sq.data_ptr(), _stream(stream)))


class BinaryCodes:
    """Hash codes on the device: codes int32 [n][dim/32] holding uint32 words (bit d = lat[d] >
    thr[d]), with the per-coordinate thresholds thr [dim] they were made with."""

    def __init__(self, lat: torch.Tensor, thr: torch.Tensor | None = None, stream=None):
        lat = lat.to(torch.float32).contiguous()
        n, dim = lat.shape
        self.fmt, self.n, self.dim = EMB_BIN, n, dim
        self.scale = self.sq = None
        if thr is None:
            thr = hash_thresholds(lat, stream)
        self.thr = thr.contiguous()
        self.codes = torch.empty((n, dim // 32), dtype=torch.int32, device=lat.device)
        _hand_to(stream, lat, self.thr, self.codes)
        _check(LIB.emb_binarize(n, dim, lat.data_ptr(), self.thr.data_ptr(), self.codes.data_ptr(),
                                _stream(stream)))


def hash_thresholds(lat: torch.Tensor, stream=None) -> torch.Tensor:
    """Per coordinate the lower median of lat [n][dim] (the database's Bi-half split)."""
    lat = lat.to(torch.float32).contiguous()
    n, dim = lat.shape
    thr = torch.empty(dim, dtype=torch.float32, device=lat.device)
    _hand_to(stream, lat, thr)
    _check(LIB.emb_hash_thresholds(n, dim, lat.data_ptr(), thr.data_ptr(), _stream(stream)))
    return thr


def emb_distances(q, x, out: torch.Tensor | None = None, stream=None):
    """[nq][n] FP32: squared L2 of quantised latents (expanded form on MFMA), or the Hamming
    distance of BinaryCodes."""
    if out is None:
        out = torch.empty((q.n, x.n), dtype=torch.float32, device=q.codes.device)
    _check(LIB.emb_distances(q.fmt, q.n, x.n, q.dim, q.codes.data_ptr(), _ptr(q.scale),
                             _ptr(q.sq), x.codes.data_ptr(), _ptr(x.scale), _ptr(x.sq),
                             out.data_ptr(), _stream(stream)))
    return out


def emb_distances_l2sum(q1, x1, q2, x2, out: torch.Tensor | None = None, stream=None):
    """[nq][n] FP32: L2(q1, x1) + L2(q2, x2), the paper's L2_T1Gd + L2_FLAIR of two encoders."""
    if out is None:
        out = torch.empty((q1.n, x1.n), dtype=torch.float32, device=q1.codes.device)
    _check(LIB.emb_distances_l2sum(q1.fmt, q1.n, x1.n, q1.dim,
                                   q1.codes.data_ptr(), _ptr(q1.scale), _ptr(q1.sq),
                                   x1.codes.data_ptr(), _ptr(x1.scale), _ptr(x1.sq),
                                   q2.codes.data_ptr(), _ptr(q2.scale), _ptr(q2.sq),
                                   x2.codes.data_ptr(), _ptr(x2.scale), _ptr(x2.sq),
                                   out.data_ptr(), _stream(stream)))
    return out


def emb_topk_min(D: torch.Tensor, k: int, stream=None, chunked: bool = True):
    """Per row the k smallest (ties by lower column), ascending: (idx int32, values). With
    chunked, rows are split over many blocks and merged (same results)."""
    M, N = D.shape
    idx = torch.empty((M, k), dtype=torch.int32, device=D.device)
    val = torch.empty((M, k), dtype=torch.float32, device=D.device)
    nb = LIB.emb_topk_min_workspace_bytes(M, N, k) if chunked else 0
    ws = torch.empty(nb, dtype=torch.uint8, device=D.device) if nb else None
    _check(LIB.emb_topk_min(M, N, D.contiguous().data_ptr(), k, idx.data_ptr(), val.data_ptr(),
                            _ptr(ws), nb, _stream(stream)))
    return idx, val


def groups_workspace(M: int, N: int, device="cuda") -> torch.Tensor:
    """Workspace shared by emb_distances_groups and emb_topk_groups for [M][N] distances."""
    return torch.empty(LIB.emb_groups_workspace_bytes(M, N), dtype=torch.uint8, device=device)


def emb_distances_groups(q, x, ws: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """emb_distances (BF16 / FP8), also leaving each row's 16-entry group minima in ws."""
    if out is None:
        out = torch.empty((q.n, x.n), dtype=torch.float32, device=q.codes.device)
    _check(LIB.emb_distances_groups(q.fmt, q.n, x.n, q.dim, q.codes.data_ptr(), _ptr(q.scale),
                                    _ptr(q.sq), x.codes.data_ptr(), _ptr(x.scale), _ptr(x.sq),
                                    out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
    return out


def emb_topk_groups(D: torch.Tensor, k: int, ws: torch.Tensor, stream=None):
    """emb_topk_min's result for D, bounded by the group minima emb_distances_groups left in ws."""
    M, N = D.shape
    idx = torch.empty((M, k), dtype=torch.int32, device=D.device)
    val = torch.empty((M, k), dtype=torch.float32, device=D.device)
    _check(LIB.emb_topk_groups(M, N, D.data_ptr(), k, idx.data_ptr(), val.data_ptr(),
                               ws.data_ptr(), ws.numel(), _stream(stream)))
    return idx, val


def knn_workspace(M: int, N: int, k: int, device="cuda") -> torch.Tensor:
    """Workspace of emb_knn for M queries, N database latents and k nearest."""
    nb = LIB.emb_knn_workspace_bytes(M, N, k)
    if nb == 0:
        raise DbError(DB_EINVAL, f"emb_knn: bad sizes M={M} N={N} k={k}")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def emb_knn(q, x, k: int, direct: bool = True, ws: torch.Tensor | None = None, out=None,
            stream=None):
    """The k nearest database latents per query in one pass (no distance matrix):
    (idx int32 [M][k], d float32 [M][k]); d in direct form unless direct=False."""
    if ws is None:
        ws = knn_workspace(q.n, x.n, k, q.codes.device)
    if out is None:
        out = (torch.empty((q.n, k), dtype=torch.int32, device=q.codes.device),
               torch.empty((q.n, k), dtype=torch.float32, device=q.codes.device))
    idx, d = out
    _check(LIB.emb_knn(q.fmt, q.n, x.n, q.dim, q.codes.data_ptr(), _ptr(q.scale), _ptr(q.sq),
                       x.codes.data_ptr(), _ptr(x.scale), _ptr(x.sq), k, 1 if direct else 0,
                       idx.data_ptr(), d.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
    return idx, d


def labels_resample(labels: torch.Tensor, shape, stream=None) -> torch.Tensor:
    """Order-0 resampling of uint8 labels [nq][nz][ny][nx] to [nq][*shape] (shape = (mz, my, mx))."""
    lab = labels.contiguous()
    if lab.dim() == 3:
        lab = lab[None]
    nq, nz, ny, nx = lab.shape
    mz, my, mx = shape
    out = torch.empty((nq, mz, my, mx), dtype=torch.uint8, device=lab.device)
    _check(LIB.labels_resample(nq, lab.data_ptr(), nx, ny, nz, out.data_ptr(), mx, my, mz,
                               _stream(stream)))
    return out
