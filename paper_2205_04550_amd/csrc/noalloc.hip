// noalloc.hip — the exact query with its workspace in a library-owned device array.
//
// db_query takes a caller workspace (the packed query, the per-entry overlaps and
// the top-k candidate lists). Callers that cannot allocate device memory at
// query time (code under HIP graph capture, tight serving loops) call
// db_query_noalloc instead: the same kernels, with the workspace carved from
// `scratch`, a fixed array in device memory that every GPU the library runs on
// holds until the process ends. Nothing here allocates.
//
// In host code `scratch` names a host-side stand-in, not the device array: the
// device address is looked up once per device with hipGetSymbolAddress (with
// that device current) and only that address is passed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = DB_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices];   // device address of `scratch` per device (null: not looked up)

// Device address of this device's copy of `scratch`; the lookup runs once per device.
hipError_t scratch_ptr(int dev, void **out)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

using namespace tdb;

extern "C" int db_query_noalloc(const db_t *db, const uint8_t *q_labels, int k, int32_t *idx,
                                double *score, db_counts_t *counts, void *stream)
{
    int rc = check_query_args("db_query_noalloc", db, q_labels, k, idx, score);
    if (rc) return rc;
    const WsLayout L = ws_layout(db, 1, k, false);
    if (L.total > kScratchBytes)
        return tdb_set_error(DB_ENOSPC,
                             "db_query_noalloc: this database needs %zu bytes of scratch, more "
                             "than the %zu the library holds (use db_query with a workspace)",
                             L.total, kScratchBytes);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return tdb_set_error(DB_EHIP, "db_query_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    if (dev != db->device || dev < 0 || dev >= kMaxDevices)
        return tdb_set_error(DB_EINVAL,
                             "db_query_noalloc: current device %d is not the database's (%d)",
                             dev, db->device);
    void *ws = nullptr;
    e = scratch_ptr(dev, &ws);
    if (e != hipSuccess)
        return tdb_set_error(DB_EHIP, "db_query_noalloc: hipGetSymbolAddress: %s",
                             hipGetErrorString(e));
    // Every piece of the workspace is written by the launches that read it (the packed
    // query up to its padding words, every overlap, every candidate list), so nothing
    // left by an earlier call needs clearing.
    e = enqueue_query(db, q_labels, k, idx, score, counts, ws, L, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return tdb_set_error(DB_EHIP, "db_query_noalloc: launch: %s", hipGetErrorString(e));
    return DB_OK;
}
