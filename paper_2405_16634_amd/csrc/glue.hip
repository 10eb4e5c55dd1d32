// Small kernels around the traversal: the Alg. 2 step length, and moving
// per-point vectors between caller order and Morton order.
#include "common.h"
#include "internal.h"

namespace wnnc {

// alpha = |r|^2 / |A r|^2 (Alg. 2) for each cloud (one workgroup per
// cloud), 0 when the denominator is 0.  The cloud's per-task partial sums
// are reduced in a fixed order.  Also stores the energy E = |rho|^2 of the
// iteration (N_c / 4 for the iteration started from mu = 0).
constexpr int kAlphaBlock = 1024;
constexpr int kAlphaUnroll = 8;

__global__ __launch_bounds__(kAlphaBlock) void k_alpha(const double *__restrict__ partial,
                                                       int nslots,
                                                       const int32_t *__restrict__ task_lo,
                                                       const int64_t *__restrict__ off, int first,
                                                       double *__restrict__ alpha,
                                                       double *__restrict__ energy_row) {
    // per thread a strided sum (kAlphaUnroll loads of each row in flight at
    // once: the loads, not the additions, set the time), per wavefront a
    // butterfly, then the wavefront sums in order: a fixed order, so the
    // result is reproducible
    constexpr int kWaves = kAlphaBlock / kWave;
    __shared__ double sh[3][kWaves];
    const int c = blockIdx.x;
    const int lo = task_lo[c], hi = task_lo[c + 1];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wv = tid / kWave;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int base = lo; base < hi; base += kAlphaUnroll * kAlphaBlock) {
        double v[3][kAlphaUnroll];
#pragma unroll
        for (int u = 0; u < kAlphaUnroll; ++u) {
            const int i = base + u * kAlphaBlock + tid;
            const int ic = i < hi ? i : hi - 1;  // in range; its value is not used
            v[0][u] = partial[ic];
            v[1][u] = partial[nslots + ic];
            v[2][u] = partial[2 * nslots + ic];
        }
#pragma unroll
        for (int u = 0; u < kAlphaUnroll; ++u) {
            if (base + u * kAlphaBlock + tid < hi) {
                if (!first) acc[0] += v[0][u];
                acc[1] += v[1][u];
                acc[2] += v[2][u];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) acc[k] += __shfl_xor(acc[k], d, kWave);
        if (lane == 0) sh[k][wv] = acc[k];
    }
    __syncthreads();
    if (tid == 0) {
        double tot[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double t = 0.0;
            for (int w = 0; w < kWaves; ++w) t += sh[k][w];
            tot[k] = t;
        }
        const double r2 = tot[1], t2 = tot[2];
        alpha[c] = t2 > 0.0 ? r2 / t2 : 0.0;
        if (energy_row) energy_row[c] = first ? 0.25 * (double)(off[c + 1] - off[c]) : tot[0];
    }
}

// out = the sum of n per-group partial sums (one workgroup; per thread a
// strided sum, then a tree over the workgroup: a fixed order)
__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ partial, int n,
                                                      double *__restrict__ out) {
    __shared__ double sh[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a += partial[i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

hipError_t launch_sum_partials(const double *partial, int n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partial, n, out);
    return hipGetLastError();
}

// flag <- 1 if any of the n floats is NaN or infinite (every writer
// stores the same value, so the race is benign)
__global__ __launch_bounds__(256) void k_check_finite(const float *__restrict__ a, int64_t n,
                                                      uint32_t *__restrict__ flag) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        bad |= !isfinite(a[i]);
    if (__ballot(bad) != 0ull && (threadIdx.x & (kWave - 1)) == 0) *flag = 1u;
}

hipError_t launch_check_finite(const float *a, int64_t n, uint32_t *flag, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256),
                       0, st, a, n, flag);
    return hipGetLastError();
}

hipError_t launch_alpha(wnnc_ctx_s *ctx, bool first, double *energy_row) {
    hipLaunchKernelGGL(k_alpha, dim3(ctx->nclouds), dim3(kAlphaBlock), 0, ctx->stream, ctx->partial.p,
                       ctx->ngroups, ctx->task_lo.p, ctx->d_offsets.p, first ? 1 : 0,
                       ctx->scalars.p, energy_row);
    return hipGetLastError();
}

// beta_c = (1/2) sum s / sum s^2 over cloud c (the least-squares uniform
// scale of the predicted normals against b = 1/2), 0 if sum s^2 = 0.
__global__ __launch_bounds__(256) void k_warm_beta(const double *__restrict__ partial, int nslots,
                                                   const int32_t *__restrict__ task_lo,
                                                   double *__restrict__ beta) {
    __shared__ double sh[2][256];
    const int c = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int i = task_lo[c] + threadIdx.x; i < task_lo[c + 1]; i += 256) {
        a += partial[i];
        b += partial[nslots + i];
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < d) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + d];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) beta[c] = sh[1][0] > 0.0 ? 0.5 * sh[0][0] / sh[1][0] : 0.0;
}

__global__ __launch_bounds__(256) void k_warm_apply(const float4 *__restrict__ nrm,
                                                    const int32_t *__restrict__ cloud,
                                                    const double *__restrict__ beta, int64_t n,
                                                    float4 *__restrict__ mu) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float b = (float)beta[cloud[i]];
    const float4 v = nrm[i];
    mu[i] = make_float4(b * v.x, b * v.y, b * v.z, 0.f);
}

hipError_t launch_warm_scale(wnnc_ctx_s *ctx, const float4 *n_sorted, float4 *mu0) {
    hipLaunchKernelGGL(k_warm_beta, dim3(ctx->nclouds), dim3(256), 0, ctx->stream, ctx->partial.p,
                       ctx->ngroups, ctx->task_lo.p, ctx->scalars.p);
    hipLaunchKernelGGL(k_warm_apply, dim3((unsigned)((ctx->n + 255) / 256)), dim3(256), 0,
                       ctx->stream, n_sorted, ctx->cloud_of.p, ctx->scalars.p, ctx->n, mu0);
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

// Per cloud, the number of points whose sorted mu points against the
// prediction nhat (caller order): mu . nhat <= 0 with mu nonzero.  One atomic
// per wavefront when its points share a cloud.
__global__ __launch_bounds__(256) void k_pred_disagree(const float4 *__restrict__ mu,
                                                       const float *__restrict__ nhat,
                                                       const uint32_t *__restrict__ perm,
                                                       const int32_t *__restrict__ cloud, int64_t n,
                                                       unsigned long long *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    int c = -1;
    if (i < n) {
        const float4 m = mu[i];
        const int64_t j = perm[i];
        const double d = (double)m.x * nhat[3 * j] + (double)m.y * nhat[3 * j + 1] +
                         (double)m.z * nhat[3 * j + 2];
        bad = (m.x != 0.f || m.y != 0.f || m.z != 0.f) && d <= 0.0;
        c = cloud[i];
    }
    const int c0 = __shfl(c, 0, 64);
    const bool same = __all(c == c0 || c < 0);
    if (same) {
        const unsigned long long k = __popcll(__ballot(bad));
        if ((threadIdx.x & 63) == 0 && k) atomicAdd(count + c0, k);
    } else if (bad) {
        atomicAdd(count + c, 1ull);
    }
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

__global__ __launch_bounds__(256) void k_gather_scalar(const float *__restrict__ src,
                                                       const uint32_t *__restrict__ perm, int64_t n,
                                                       float *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

hipError_t launch_gather_scalar(const float *src, const uint32_t *perm, float *dst, int64_t n,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_gather_scalar, dim3(nblk(n)), dim3(256), 0, st, src, perm, n, dst);
    return hipGetLastError();
}

hipError_t launch_pred_disagree(wnnc_ctx_s *ctx, const float4 *mu, const float *nhat,
                                unsigned long long *count) {
    hipLaunchKernelGGL(k_pred_disagree, dim3(nblk(ctx->n)), dim3(256), 0, ctx->stream, mu, nhat,
                       ctx->perm.p, ctx->cloud_of.p, ctx->n, count);
    return hipGetLastError();
}

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
