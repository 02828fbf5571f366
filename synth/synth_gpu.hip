/*
 * synth_gpu.hip — seeded synthetic inputs, GPU build of synth_formula.h.
 *
 * Writes the same float32 concentration volumes as synth_fill_cpu(), but on
 * the device, so that a 50,000 x 128^3 database (419 GB of float32) can be
 * produced chunk by chunk in HBM instead of over PCIe. Parameters come from
 * the host-side synth_params() (same seed => same table). Input generator
 * only; not part of the retrieval library.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "synth_formula.h"

// grid (ny * nz rows, simulations): one block fills one x-row of one volume.
__global__ void __launch_bounds__(128) synth_fill_kernel(const synth_params_t *__restrict__ params,
                                                         synth_brain_t b, int nx, int ny, int nz,
                                                         float *__restrict__ out)
{
    const int r = blockIdx.x;
    const int t = blockIdx.y;
    const int j = r % ny;
    const int k = r / ny;
    const synth_params_t p = params[t];
    float *o = out + ((int64_t)t * nz * ny + r) * nx;
    for (int i = threadIdx.x; i < nx; i += blockDim.x)
        o[i] = synth_conc(&p, &b, i, j, k);
}

extern "C" int synth_fill_gpu(const void *params_dev, int64_t count, int nx, int ny, int nz,
                              float *out_dev, void *stream)
{
    if (count <= 0) return 0;
    if (!params_dev || !out_dev || nx <= 0 || ny <= 0 || nz <= 0) return -1;
    synth_brain_t b;
    b.Cx = (nx - 1) * 0.5;
    b.Cy = (ny - 1) * 0.5;
    b.Cz = (nz - 1) * 0.5;
    b.iAx = 1.0 / (0.40 * nx);
    b.iAy = 1.0 / (0.46 * ny);
    b.iAz = 1.0 / (0.36 * nz);
    if ((int64_t)ny * nz > 0x7fffffff) return -1;
    const int64_t V = (int64_t)nx * ny * nz;
    for (int64_t t0 = 0; t0 < count; t0 += 65535) {
        const int64_t c = (count - t0 < 65535) ? count - t0 : 65535;
        hipLaunchKernelGGL(synth_fill_kernel, dim3((unsigned)(ny * nz), (unsigned)c), dim3(128), 0,
                           (hipStream_t)stream, (const synth_params_t *)params_dev + t0, b, nx, ny,
                           nz, out_dev + t0 * V);
        if (hipGetLastError() != hipSuccess) return -2;
    }
    return 0;
}
