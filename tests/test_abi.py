"""The C ABI library loads, exports what include/tumordb.h declares, and rejects bad
arguments before touching the GPU (CPU-only checks)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("tumordb.h", "tumornn.h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b((?:db|emb|nn|labels)_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("db_build", "db_append", "db_query", "db_query_batch", "db_scan", "db_sync",
              "db_free", "db_last_error", "db_storage_bytes", "db_query_workspace_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2205_04550_amd import binding, nn
    lib = ctypes.CDLL(binding.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    # The Python binding covers exactly the declared C entry points.
    assert set(declared_functions()) == set(binding.SYMBOLS) | set(nn.NN_SYMBOLS)


def test_storage_bytes():
    from paper_2205_04550_amd import binding
    # 128^3: 65,536 words per mask plane, 2 planes, 4 bytes; popcounts 8 bytes per entry;
    # row boxes 16, moments 32, the tile order 4, the T1Gd row boxes 16, the per-slice
    # y-ranges 8 nz bytes and the 16^3-block counts 2 masks x 512 blocks x 2 bytes per entry;
    # each piece 256-byte aligned.
    up = lambda b: (b + 255) // 256 * 256
    planes = 50000 * 2 * 65536 * 4
    meta = (up(50000 * 8) + up(50000 * 16) + up(50000 * 32) + up(50000 * 4) + up(50000 * 16) +
            up(50000 * 128 * 8) + up(50000 * 2 * 512 * 2))
    assert binding.storage_bytes(128, 128, 128, 50000) == planes + meta
    # Ragged plane: 32x3x1 = 3 words, padded to 4: 10*2*4*4 = 320 -> 512; then 80, 160,
    # 320, 40, 160 and 80 bytes -> 256, 256, 512, 256, 256 and 256; 2 x 1 x 1 blocks padded
    # to 8: 10*2*8*2 = 320 -> 512.
    assert binding.storage_bytes(32, 3, 1, 10) == 512 + 256 + 256 + 512 + 256 + 256 + 256 + 512
    # 512^3: 32^3 blocks, more than the bound keeps: no block counts.
    assert binding.storage_bytes(512, 512, 512, 1) == (
        up(2 * 512 ** 3 // 8) + 256 * 5 + up(512 * 8))
    assert binding.storage_bytes(33, 4, 4, 10) == 0      # nx not a multiple of 32
    assert binding.storage_bytes(32, 0, 4, 10) == 0
    assert binding.storage_bytes(32, 4, 4, 0) == 0


def test_build_rejects_bad_arguments_before_any_gpu_call():
    from paper_2205_04550_amd import binding as b
    h = ctypes.c_void_p()
    assert b.LIB.db_build(None, 64, 64, 64, 0.25, 0.675, 10, 256, 1 << 30) == b.DB_EINVAL
    assert b"NULL" in b.LIB.db_last_error()
    assert b.LIB.db_build(ctypes.byref(h), 63, 64, 64, 0.25, 0.675, 10, 256, 1 << 30) == b.DB_EINVAL
    assert b.LIB.db_build(ctypes.byref(h), 64, 64, 64, 0.7, 0.25, 10, 256, 1 << 30) == b.DB_EINVAL
    assert b.LIB.db_build(ctypes.byref(h), 64, 64, 64, 0.25, 0.675, 10, None, 1 << 30) == b.DB_EINVAL
    assert b.LIB.db_build(ctypes.byref(h), 64, 64, 64, 0.25, 0.675, 10, 257, 1 << 30) == b.DB_EINVAL
    assert b.LIB.db_build(ctypes.byref(h), 64, 64, 64, 0.25, 0.675, 10, 256, 100) == b.DB_ENOSPC
    assert b"needed" in b.LIB.db_last_error()
    assert h.value is None


def test_calls_on_invalid_handle():
    from paper_2205_04550_amd import binding as b
    assert b.LIB.db_size(None) == -1
    assert b.LIB.db_query(None, 256, 1, 256, 256, None, 256, 1 << 20, None) == b.DB_ESTATE
    assert b.LIB.db_query_batch(None, 1, 256, None, 1, 256, 256, None, 256, 1 << 20, None) == b.DB_ESTATE
    assert b.LIB.db_scan(None, 256, 256, None, 256, 1 << 20, None) == b.DB_ESTATE
    assert b.LIB.db_append(None, 256, 1, None) == b.DB_ESTATE
    assert b.LIB.db_sync(None, None) == b.DB_ESTATE
    assert b.LIB.db_query_workspace_bytes(None, 1, 10) == 0
    b.LIB.db_free(None)  # no-op


def test_group_path_sizes_and_argument_errors_before_any_gpu_call():
    from paper_2205_04550_amd import binding as b
    # tau (M words, 256-byte aligned) + the group minima [M][N / 16] (whole groups only).
    assert b.LIB.emb_groups_workspace_bytes(1024, 50_000) == 4096 + 1024 * 3125 * 4
    assert b.LIB.emb_groups_workspace_bytes(3, 50_021) == 256 + 3 * 3126 * 4
    assert b.LIB.emb_groups_workspace_bytes(0, 100) == 0
    fake = 1 << 20                                  # aligned non-null pointers, never dereferenced
    assert b.LIB.emb_topk_groups(4, 100, None, 5, fake, fake, fake, 1 << 20, None) == b.DB_EINVAL
    assert b.LIB.emb_topk_groups(4, 100, fake, 101, fake, fake, fake, 1 << 20, None) == b.DB_EINVAL
    assert b.LIB.emb_topk_groups(4, 100, fake, 5, fake, fake, None, 1 << 20, None) == b.DB_ENOSPC
    assert b.LIB.emb_topk_groups(4, 100, fake, 5, fake, fake, fake, 16, None) == b.DB_ENOSPC
    sq = fake
    assert b.LIB.emb_distances_groups(b.EMB_BIN, 4, 100, 64, fake, None, None, fake, None, None,
                                      fake, fake, 1 << 20, None) == b.DB_EINVAL
    assert b.LIB.emb_distances_groups(b.EMB_BF16, 4, 100, 64, fake, None, sq, fake, None, sq,
                                      fake, fake, 16, None) == b.DB_ENOSPC
    assert b"needed" in b.LIB.db_last_error()
    # Query codes of 2 GiB or more are refused (32-bit row offsets in the distance kernel).
    assert b.LIB.emb_distances(b.EMB_BF16, 1 << 20, 100, 1024, fake, None, sq, fake, None, sq,
                               fake, None) == b.DB_EINVAL
