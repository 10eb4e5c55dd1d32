// The neighbourhood MLP of the learned warm start: 48 -> 64 -> 64 -> 3 with
// ReLU, BF16 operands and FP32 accumulation, inference and training.
//
// Every product is one generic GEMM kernel on the CDNA4 matrix cores
// (v_mfma_f32_16x16x32_bf16): one wavefront computes a 16x16 tile of
// C = A B over a range of K in steps of 32, with A and B read from FP32
// memory through strides (so transposes cost nothing), rounded to BF16 (round
// to nearest even) when the fragments are formed.  Lane l holds
// A[l%16][8(l/16)+i] and B[8(l/16)+i][l%16], i = 0..7, and receives
// C[4(l/16)+i][l%16], i = 0..3.  Long reductions (weight gradients, K = batch
// size) are split over workgroups into partial tiles that a second kernel
// adds in a fixed order, so training is reproducible bit for bit.
//
// Parameter vector (FP32 master copy, 7491 values): W1 [48][64], b1 [64],
// W2 [64][64], b2 [64], W3 [64][3], b3 [3]; row-major [in][out].
#include <float.h>

#include "common.h"
#include "internal.h"

namespace wnnc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ inline __bf16 to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __builtin_bit_cast(__bf16, (unsigned short)(u >> 16));
}

struct GemmArgs {
    const float *A;
    int64_t sam, sak;  // A(m,k) = A[m*sam + k*sak]
    const float *B;
    int64_t sbk, sbn;  // B(k,n) = B[k*sbk + n*sbn]
    float *C;
    int64_t ldc;       // C(m,n) = C[split*split_stride + m*ldc + n]
    int64_t split_stride;
    int M, N, K;
    int k_per_split;   // multiple of 32
    const float *bias; // epilogue: + bias[n]
    int relu;          // epilogue: max(., 0)
    const float *mask; // epilogue: zero where mask(m,n) <= 0 (same layout as C)
};

__global__ __launch_bounds__(64) void k_gemm(GemmArgs g) {
    const int l = threadIdx.x;
    const int r = l & 15, q = l >> 4;
    const int m0 = blockIdx.x * 16, n0 = blockIdx.y * 16;
    const int kb = blockIdx.z * g.k_per_split;
    const int ke = min(g.K, kb + g.k_per_split);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int am = m0 + r, bn = n0 + r;
    for (int k0 = kb; k0 < ke; k0 += 32) {
        bf16x8 a, b;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = k0 + 8 * q + i;
            const bool kin = k < ke;
            const float av = (kin && am < g.M) ? g.A[am * g.sam + k * g.sak] : 0.0f;
            const float bv = (kin && bn < g.N) ? g.B[k * g.sbk + bn * g.sbn] : 0.0f;
            a[i] = to_bf16(av);
            b[i] = to_bf16(bv);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    float *C = g.C + (int64_t)blockIdx.z * g.split_stride;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + 4 * q + i, n = n0 + r;
        if (m >= g.M || n >= g.N) continue;
        float v = acc[i];
        if (g.bias) v += g.bias[n];
        if (g.relu) v = fmaxf(v, 0.0f);
        if (g.mask && !(g.mask[(int64_t)m * g.ldc + n] > 0.0f)) v = 0.0f;
        C[(int64_t)m * g.ldc + n] = v;
    }
}

// out[i] = sum over splits s of part[s * stride + i], in order
__global__ __launch_bounds__(256) void k_split_sum(const float *__restrict__ part, int splits,
                                                   int64_t stride, int64_t count,
                                                   float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.0f;
    for (int k = 0; k < splits; ++k) s += part[k * stride + i];
    out[i] = s;
}

// column sums of an (rows x cols) row-major matrix, one workgroup per column
__global__ __launch_bounds__(256) void k_colsum(const float *__restrict__ X, int64_t rows, int cols,
                                                float *__restrict__ out) {
    __shared__ float sh[256];
    const int c = blockIdx.x;
    float s = 0.0f;
    for (int64_t i = threadIdx.x; i < rows; i += 256) s += X[i * cols + c];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sh[0];
}

// loss = mean_i (1 - cos(y_i, l_i)); dy = d loss / d y.  Per-block partial
// loss sums (FP64) are reduced in order on the host side of the call.
__global__ __launch_bounds__(256) void k_cos_loss(const float *__restrict__ Y,
                                                  const float *__restrict__ L, int64_t n,
                                                  float inv_n, float *__restrict__ dY,
                                                  double *__restrict__ part) {
    __shared__ double sh[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double loss = 0.0;
    if (i < n) {
        const float y0 = Y[3 * i], y1 = Y[3 * i + 1], y2 = Y[3 * i + 2];
        const float l0 = L[3 * i], l1 = L[3 * i + 1], l2 = L[3 * i + 2];
        const float yy = sqrtf(y0 * y0 + y1 * y1 + y2 * y2);
        const float ll = sqrtf(l0 * l0 + l1 * l1 + l2 * l2);
        float d0 = 0.f, d1 = 0.f, d2 = 0.f;
        float cs = 0.f;
        if (yy > 0.f && ll > 0.f) {
            const float yl = y0 * l0 + y1 * l1 + y2 * l2;
            cs = yl / (yy * ll);
            // d cos / d y = l/(|y||l|) - (y.l) y / (|y|^3 |l|)
            const float a = 1.0f / (yy * ll), b = yl / (yy * yy * yy * ll);
            d0 = -inv_n * (l0 * a - y0 * b);
            d1 = -inv_n * (l1 * a - y1 * b);
            d2 = -inv_n * (l2 * a - y2 * b);
        }
        loss = 1.0 - (double)cs;
        dY[3 * i] = d0, dY[3 * i + 1] = d1, dY[3 * i + 2] = d2;
    }
    sh[threadIdx.x] = loss;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_unit_rows(const float *__restrict__ Y, int64_t n,
                                                   float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float y0 = Y[3 * i], y1 = Y[3 * i + 1], y2 = Y[3 * i + 2];
    const float yy = sqrtf(y0 * y0 + y1 * y1 + y2 * y2);
    const float f = yy > 0.f ? 1.0f / yy : 0.0f;
    out[3 * i] = y0 * f, out[3 * i + 1] = y1 * f, out[3 * i + 2] = y2 * f;
}

// Adam on the FP32 master parameters (bias-corrected moments).
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, float *__restrict__ m,
                                              float *__restrict__ v,
                                              const float *__restrict__ g, int count, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------ host --

namespace {

void gemm(hipStream_t st, const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk,
          int64_t sbn, float *C, int64_t ldc, int M, int N, int K, const float *bias, bool relu,
          const float *mask, int splits = 1, int64_t split_stride = 0) {
    GemmArgs g;
    g.A = A, g.sam = sam, g.sak = sak;
    g.B = B, g.sbk = sbk, g.sbn = sbn;
    g.C = C, g.ldc = ldc, g.split_stride = split_stride;
    g.M = M, g.N = N, g.K = K;
    int kps = (K + splits - 1) / splits;
    kps = (kps + 31) / 32 * 32;
    g.k_per_split = kps;
    g.bias = bias, g.relu = relu ? 1 : 0, g.mask = mask;
    const dim3 grid((unsigned)((M + 15) / 16), (unsigned)((N + 15) / 16), (unsigned)splits);
    hipLaunchKernelGGL(k_gemm, grid, dim3(64), 0, st, g);
}

// a weight gradient C (M x N, ldc = N) = A^T-like product with K = rows,
// split over workgroups and summed in order
hipError_t gemm_split(wnnc_ctx_s *ctx, const float *A, int64_t sam, int64_t sak, const float *B,
                      int64_t sbk, int64_t sbn, float *C, int M, int N, int K) {
    int splits = (K + 2047) / 2048;
    if (splits > 512) splits = 512;
    if (splits < 1) splits = 1;
    const int64_t stride = (int64_t)M * N;
    hipError_t e = ctx->mlp_part.ensure(stride * splits);
    if (e != hipSuccess) return e;
    gemm(ctx->stream, A, sam, sak, B, sbk, sbn, ctx->mlp_part.p, N, M, N, K, nullptr, false,
         nullptr, splits, stride);
    hipLaunchKernelGGL(k_split_sum, dim3((unsigned)((stride + 255) / 256)), dim3(256), 0,
                       ctx->stream, ctx->mlp_part.p, splits, stride, stride, C);
    return hipGetLastError();
}

}  // namespace

hipError_t mlp_forward(wnnc_ctx_s *ctx, const float *P, const float *X, int64_t n, float *Y) {
    hipStream_t st = ctx->stream;
    hipError_t e = ctx->mlp_h1.ensure(n * kMlpHidden);
    if (e == hipSuccess) e = ctx->mlp_h2.ensure(n * kMlpHidden);
    if (e != hipSuccess) return e;
    float *H1 = ctx->mlp_h1.p, *H2 = ctx->mlp_h2.p;
    const int N = (int)n;
    gemm(st, X, kMlpIn, 1, P + kOffW1, kMlpHidden, 1, H1, kMlpHidden, N, kMlpHidden, kMlpIn,
         P + kOffB1, true, nullptr);
    gemm(st, H1, kMlpHidden, 1, P + kOffW2, kMlpHidden, 1, H2, kMlpHidden, N, kMlpHidden,
         kMlpHidden, P + kOffB2, true, nullptr);
    gemm(st, H2, kMlpHidden, 1, P + kOffW3, kMlpOut, 1, Y, kMlpOut, N, kMlpOut, kMlpHidden,
         P + kOffB3, false, nullptr);
    return hipGetLastError();
}

hipError_t mlp_normals(wnnc_ctx_s *ctx, const float *Y, int64_t n, float *out) {
    hipLaunchKernelGGL(k_unit_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, Y,
                       n, out);
    return hipGetLastError();
}

hipError_t mlp_loss_grad(wnnc_ctx_s *ctx, const float *P, const float *X, const float *L,
                         int64_t n, float *grad, double *loss) {
    hipStream_t st = ctx->stream;
    hipError_t e = ctx->mlp_y.ensure(n * kMlpOut);
    if (e == hipSuccess) e = ctx->mlp_dy.ensure(n * kMlpOut);
    if (e == hipSuccess) e = ctx->mlp_d2.ensure(n * kMlpHidden);
    if (e == hipSuccess) e = ctx->mlp_d1.ensure(n * kMlpHidden);
    const int64_t nb = (n + 255) / 256;
    if (e == hipSuccess) e = ctx->mlp_lpart.ensure(nb);
    if (e != hipSuccess) return e;
    e = mlp_forward(ctx, P, X, n, ctx->mlp_y.p);
    if (e != hipSuccess) return e;
    float *H1 = ctx->mlp_h1.p, *H2 = ctx->mlp_h2.p, *Y = ctx->mlp_y.p, *dY = ctx->mlp_dy.p;
    float *D2 = ctx->mlp_d2.p, *D1 = ctx->mlp_d1.p;
    const int N = (int)n;
    hipLaunchKernelGGL(k_cos_loss, dim3((unsigned)nb), dim3(256), 0, st, Y, L, n, 1.0f / (float)n,
                       dY, ctx->mlp_lpart.p);
    // layer 3: dW3 = H2^T dY, db3 = colsum dY, dH2 = (dY W3^T) * [H2 > 0]
    e = gemm_split(ctx, H2, 1, kMlpHidden, dY, kMlpOut, 1, grad + kOffW3, kMlpHidden, kMlpOut, N);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3(kMlpOut), dim3(256), 0, st, dY, n, kMlpOut, grad + kOffB3);
    gemm(st, dY, kMlpOut, 1, P + kOffW3, 1, kMlpOut, D2, kMlpHidden, N, kMlpHidden, kMlpOut,
         nullptr, false, H2);
    // layer 2
    e = gemm_split(ctx, H1, 1, kMlpHidden, D2, kMlpHidden, 1, grad + kOffW2, kMlpHidden,
                   kMlpHidden, N);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3(kMlpHidden), dim3(256), 0, st, D2, n, kMlpHidden,
                       grad + kOffB2);
    gemm(st, D2, kMlpHidden, 1, P + kOffW2, 1, kMlpHidden, D1, kMlpHidden, N, kMlpHidden,
         kMlpHidden, nullptr, false, H1);
    // layer 1
    e = gemm_split(ctx, X, 1, kMlpIn, D1, kMlpHidden, 1, grad + kOffW1, kMlpIn, kMlpHidden, N);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3(kMlpHidden), dim3(256), 0, st, D1, n, kMlpHidden,
                       grad + kOffB1);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (loss) {
        std::vector<double> lp((size_t)nb);
        e = hipMemcpyAsync(lp.data(), ctx->mlp_lpart.p, (size_t)nb * sizeof(double),
                           hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        double s = 0.0;
        for (double v : lp) s += v;
        *loss = s / (double)n;
    }
    return hipSuccess;
}

hipError_t mlp_adam(wnnc_ctx_s *ctx, float *P, float *m, float *v, const float *g, int step,
                    float lr, float b1, float b2, float eps) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, ctx->stream, P, m, v,
                       g, kMlpParams, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace wnnc
