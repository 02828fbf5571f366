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

__global__ void __launch_bounds__(256) synth_fill_kernel(const synth_params_t *__restrict__ params,
                                                         synth_brain_t b, int nx, int ny, int nz,
                                                         int64_t total, float *__restrict__ out)
{
    int64_t V = (int64_t)nx * ny * nz;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        int64_t t = g / V;
        int64_t v = g - t * V;
        int i = (int)(v % nx);
        int64_t r = v / nx;
        int j = (int)(r % ny);
        int k = (int)(r / ny);
        synth_params_t p = params[t];
        out[g] = synth_conc(&p, &b, i, j, k);
    }
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
    int64_t total = count * (int64_t)nx * ny * nz;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(synth_fill_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, (const synth_params_t *)params_dev, b, nx, ny, nz,
                       total, out_dev);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
