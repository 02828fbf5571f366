// vae.hip — the variational head of the paper's VAE variant (Sec. 2.3,
// "Autoencoders"; Sec. 2.4: the linear layer before the latent is replaced by
// two linear layers giving the mean and the log-variance).
//
// The encoder's last linear layer writes ML [B][2L]: row b holds mu_b (L
// values) then logvar_b (L values). Training samples z = mu + exp(logvar / 2)
// * eps with eps ~ N(0, 1) passed in, and adds beta * KL to the
// reconstruction loss, KL = (1/B) sum_b sum_d -1/2 (1 + logvar - mu^2 -
// exp(logvar)), the divergence of N(mu, exp(logvar)) from N(0, 1) (the
// standard VAE objective the paper cites). Retrieval uses mu.
#include <hip/hip_runtime.h>

#include "../../include/tumornn.h"
#include "internal.hpp"

namespace tdb {

constexpr int kKlBlocks = 256;

template <typename T>
__global__ void __launch_bounds__(256) vae_fwd_kernel(int B, int L, const T *__restrict__ ML,
                                                      const T *__restrict__ eps, T *__restrict__ z,
                                                      T *__restrict__ part)
{
    __shared__ T red[256];
    const int64_t total = (int64_t)B * L;
    T acc = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t / L, d = t - b * L;
        const T mu = ML[b * 2 * L + d], lv = ML[b * 2 * L + L + d];
        const T sd = exp(T(0.5) * lv);
        z[t] = mu + sd * eps[t];
        acc += (T(1) + lv - mu * mu) - exp(lv);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// One block: the partial sums in block order, then KL = -1/2 * sum / B.
template <typename T>
__global__ void __launch_bounds__(256) kl_final_kernel(int B, const T *__restrict__ part, int np,
                                                       T *__restrict__ kl)
{
    __shared__ T red[256];
    T acc = 0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) kl[0] = T(-0.5) * red[0] / T(B);
}

// d mu = dz + beta * mu / B
// d logvar = dz * eps * exp(logvar / 2) / 2 + beta * (exp(logvar) - 1) / (2 B)
template <typename T>
__global__ void __launch_bounds__(256) vae_bwd_kernel(int B, int L, T beta, const T *__restrict__ ML,
                                                      const T *__restrict__ eps,
                                                      const T *__restrict__ dz,
                                                      T *__restrict__ dML)
{
    const int64_t total = (int64_t)B * L;
    const T inv2b = T(0.5) / T(B);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t / L, d = t - b * L;
        const T mu = ML[b * 2 * L + d], lv = ML[b * 2 * L + L + d];
        const T g = dz[t];
        dML[b * 2 * L + d] = g + beta * mu / T(B);
        dML[b * 2 * L + L + d] = g * eps[t] * T(0.5) * exp(T(0.5) * lv) + beta * (exp(lv) - T(1)) * inv2b;
    }
}

}  // namespace tdb

using namespace tdb;

namespace {

int vae_launched(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return tdb_set_error(DB_EHIP, "%s: %s", what, hipGetErrorString(e));
    return DB_OK;
}

unsigned vae_grid(int64_t n)
{
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

extern "C" {

size_t nn_vae_ws_bytes(int dtype, int B, int L)
{
    if ((dtype != NN_F32 && dtype != NN_F64) || B <= 0 || L <= 0) return 0;
    return (size_t)kKlBlocks * (dtype == NN_F64 ? 8 : 4);
}

int nn_vae_head_fwd(int dtype, int B, int L, const void *ML, const void *eps, void *z, void *kl,
                    void *ws, size_t ws_bytes, void *stream)
{
    if ((dtype != NN_F32 && dtype != NN_F64) || B <= 0 || L <= 0 || !ML || !eps || !z || !kl ||
        !ws)
        return tdb_set_error(DB_EINVAL, "nn_vae_head_fwd: bad arguments");
    if (ws_bytes < nn_vae_ws_bytes(dtype, B, L))
        return tdb_set_error(DB_ENOSPC, "nn_vae_head_fwd: workspace %zu bytes too small", ws_bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == NN_F64) {
        hipLaunchKernelGGL(vae_fwd_kernel<double>, dim3(kKlBlocks), dim3(256), 0, s, B, L,
                           (const double *)ML, (const double *)eps, (double *)z, (double *)ws);
        hipLaunchKernelGGL(kl_final_kernel<double>, dim3(1), dim3(256), 0, s, B, (const double *)ws,
                           kKlBlocks, (double *)kl);
    } else {
        hipLaunchKernelGGL(vae_fwd_kernel<float>, dim3(kKlBlocks), dim3(256), 0, s, B, L,
                           (const float *)ML, (const float *)eps, (float *)z, (float *)ws);
        hipLaunchKernelGGL(kl_final_kernel<float>, dim3(1), dim3(256), 0, s, B, (const float *)ws,
                           kKlBlocks, (float *)kl);
    }
    return vae_launched("nn_vae_head_fwd");
}

int nn_vae_head_bwd(int dtype, int B, int L, double beta, const void *ML, const void *eps,
                    const void *dz, void *dML, void *stream)
{
    if ((dtype != NN_F32 && dtype != NN_F64) || B <= 0 || L <= 0 || !ML || !eps || !dz || !dML)
        return tdb_set_error(DB_EINVAL, "nn_vae_head_bwd: bad arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const unsigned g = vae_grid((int64_t)B * L);
    if (dtype == NN_F64)
        hipLaunchKernelGGL(vae_bwd_kernel<double>, dim3(g), dim3(256), 0, s, B, L, beta,
                           (const double *)ML, (const double *)eps, (const double *)dz,
                           (double *)dML);
    else
        hipLaunchKernelGGL(vae_bwd_kernel<float>, dim3(g), dim3(256), 0, s, B, L, (float)beta,
                           (const float *)ML, (const float *)eps, (const float *)dz, (float *)dML);
    return vae_launched("nn_vae_head_bwd");
}

}  // extern "C"
