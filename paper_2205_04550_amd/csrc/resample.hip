// resample.hip — order-0 (nearest-neighbour) resampling of packed masks and query labels.
//
// Paper Sec. 2.3: the simplest speed-up the paper tries is to shrink every
// volume to 64^3 or 32^3 with an order-0 spline and run the same Dice query
// on the smaller grid (DS64 / DS32 in Tables 1 and 2). Order 0 picks
// one source voxel per output voxel, so thresholding commutes with it and the
// packed masks can be resampled directly. Output voxel o of an axis reads
// source voxel round(o * (n_in - 1) / (n_out - 1)): the output samples are
// spread evenly from the first to the last source voxel (the convention of
// the order-0 zoom the paper used); that ratio never lands on a half, so the
// rounding has no ties.
#include "common.hpp"
#include "internal.hpp"

namespace tdb {

// One block per output entry: word w of each output mask gathers 32 source bits.
__global__ void __launch_bounds__(256) resample_db_kernel(const uint32_t *__restrict__ src,
                                                          int Wp_s, int nxw_s, int ny_s,
                                                          uint32_t *__restrict__ dst, int W_d,
                                                          int Wp_d, int nxw_d, int ny_d,
                                                          uint32_t *__restrict__ pc_d,
                                                          ResampleMaps maps)
{
    __shared__ uint32_t red[2 * 4];
    const int64_t e = blockIdx.x;
    const uint32_t *s0 = src + e * 2 * (int64_t)Wp_s, *s1 = s0 + Wp_s;
    uint32_t *o = dst + e * 2 * (int64_t)Wp_d;
    uint32_t n0 = 0, n1 = 0;
    for (int w = threadIdx.x; w < Wp_d; w += blockDim.x) {
        uint32_t b0 = 0, b1 = 0;
        if (w < W_d) {
            const int wx = w % nxw_d, row = w / nxw_d;
            const int y = row % ny_d, z = row / ny_d;
            const int64_t base = ((int64_t)maps.z[z] * ny_s + maps.y[y]) * nxw_s;
            for (int b = 0; b < 32; ++b) {
                const int sx = maps.x[32 * wx + b];
                b0 |= ((s0[base + (sx >> 5)] >> (sx & 31)) & 1u) << b;
                b1 |= ((s1[base + (sx >> 5)] >> (sx & 31)) & 1u) << b;
            }
        }
        o[w] = b0;
        o[Wp_d + w] = b1;
        n0 += popc(b0);
        n1 += popc(b1);
    }
    block_sum2(n0, n1, red);
    if (threadIdx.x == 0) {
        pc_d[2 * e] = n0;
        pc_d[2 * e + 1] = n1;
    }
}

// out[q][z][y][x] = in[q][mz[z]][my[y]][mx[x]].
__global__ void resample_labels_kernel(const uint8_t *__restrict__ in, int nx, int ny, int nz,
                                       uint8_t *__restrict__ out, int mx, int my, int mz, int nq,
                                       ResampleMaps maps)
{
    const int64_t per = (int64_t)mx * my * mz;
    const int64_t total = per * nq;
    const int64_t vin = (int64_t)nx * ny * nz;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = t / per;
        int64_t r = t - q * per;
        const int x = (int)(r % mx);
        r /= mx;
        const int y = (int)(r % my);
        const int z = (int)(r / my);
        out[t] = in[q * vin + ((int64_t)maps.z[z] * ny + maps.y[y]) * nx + maps.x[x]];
    }
}

hipError_t launch_resample_db(const db_t *src, int64_t first, int64_t n, db_t *dst,
                              const ResampleMaps &maps, hipStream_t s)
{
    const Geometry &gs = src->g, &gd = dst->g;
    hipLaunchKernelGGL(resample_db_kernel, dim3((unsigned)n), dim3(256), 0, s,
                       src->planes + first * 2 * (int64_t)gs.Wp, gs.Wp, gs.nxw, gs.ny,
                       dst->planes + dst->count * 2 * (int64_t)gd.Wp, gd.W, gd.Wp, gd.nxw, gd.ny,
                       dst->popcnt + dst->count * 2, maps);
    return hipGetLastError();
}

hipError_t launch_resample_labels(int nq, const uint8_t *in, int nx, int ny, int nz, uint8_t *out,
                                  int mx, int my, int mz, const ResampleMaps &maps, hipStream_t s)
{
    int64_t total = (int64_t)nq * mx * my * mz;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(resample_labels_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, nx, ny,
                       nz, out, mx, my, mz, nq, maps);
    return hipGetLastError();
}

}  // namespace tdb
