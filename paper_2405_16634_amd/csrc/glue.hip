// Small kernels around the traversal: the Alg. 2 step length, and moving
// per-point vectors between caller order and Morton order.
#include "common.h"
#include "internal.h"

namespace wnnc {

// alpha = |r|^2 / |A r|^2 (Alg. 2), 0 when the denominator is 0.  The
// per-block partial sums are reduced in a fixed order.  Also stores the
// energy E = |rho|^2 of the iteration (or e_const when >= 0).
__global__ __launch_bounds__(256) void k_alpha(const double *__restrict__ partial, int nb,
                                               double e_const, double *__restrict__ scalars,
                                               double *__restrict__ energy_slot) {
    __shared__ double sh[3][256];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nb; i += 256) {
        if (e_const < 0.0) acc[0] += partial[i];
        acc[1] += partial[nb + i];
        acc[2] += partial[2 * nb + i];
    }
    for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < d)
            for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double r2 = sh[1][0], t2 = sh[2][0];
        scalars[0] = t2 > 0.0 ? r2 / t2 : 0.0;
        if (energy_slot) energy_slot[0] = e_const >= 0.0 ? e_const : sh[0][0];
    }
}

hipError_t launch_alpha(wnnc_ctx_s *ctx, int nb, double e_const, double *energy_slot) {
    hipLaunchKernelGGL(k_alpha, dim3(1), dim3(256), 0, ctx->stream, ctx->partial.p, nb, e_const,
                       ctx->scalars.p, energy_slot);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero_f4(float4 *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ __launch_bounds__(256) void k_gather_vec(const float *__restrict__ src,
                                                    const uint32_t *__restrict__ perm,
                                                    float4 *__restrict__ dst, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    dst[i] = make_float4(src[3 * j], src[3 * j + 1], src[3 * j + 2], 0.f);
}

__global__ __launch_bounds__(256) void k_scatter_vec(const float4 *__restrict__ src,
                                                     const uint32_t *__restrict__ perm,
                                                     float *__restrict__ dst, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    const float4 v = src[i];
    dst[3 * j] = v.x;
    dst[3 * j + 1] = v.y;
    dst[3 * j + 2] = v.z;
}

__global__ __launch_bounds__(256) void k_normals(const float *mu, int64_t n, float inv_s2,
                                                 float *nrm, float *area) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = mu[3 * i], y = mu[3 * i + 1], z = mu[3 * i + 2];
    const double l2 = (double)x * x + (double)y * y + (double)z * z;
    const double l = sqrt(l2);
    const float f = l > 0.0 ? (float)(1.0 / l) : 0.0f;
    nrm[3 * i] = x * f;
    nrm[3 * i + 1] = y * f;
    nrm[3 * i + 2] = z * f;
    if (area) area[i] = (float)(l * inv_s2);
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_zero_f4(float4 *p, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_f4, dim3(nblk(n)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_gather_vec(const float *src, const uint32_t *perm, float4 *dst, int64_t n,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_gather_vec, dim3(nblk(n)), dim3(256), 0, st, src, perm, dst, n);
    return hipGetLastError();
}

hipError_t launch_scatter_vec(const float4 *src, const uint32_t *perm, float *dst, int64_t n,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_scatter_vec, dim3(nblk(n)), dim3(256), 0, st, src, perm, dst, n);
    return hipGetLastError();
}

hipError_t launch_normals(const float *mu, int64_t n, double scale, float *nrm, float *area,
                          hipStream_t st) {
    const float inv_s2 = (float)(1.0 / (scale * scale));
    hipLaunchKernelGGL(k_normals, dim3(nblk(n)), dim3(256), 0, st, mu, n, inv_s2, nrm, area);
    return hipGetLastError();
}

}  // namespace wnnc
