// Throughput probes for one GPU's vector ALU and HBM.
//
// Each probe kernel issues a known number of one kind of vector instruction
// (kChains independent dependency chains per lane, `iters` steps each), or
// moves a known number of bytes, so that the elapsed time of a launch gives
// the chip's rate for that kind.  The figures ground the ceilings that the
// traversal's roofline is priced against: the wave64 issue rate of FP32 FMA,
// the rate of the hardware reciprocal square root (one per pair term), of
// FP64 adds and FP32 -> FP64 conversions (the per-target FP64 sums), and the
// HBM bandwidth a plain stream reaches.
//
// C ABI: wnnc_rates_run(kind, blocks, iters, out, ms_out) launches the probe
// `kind` once untimed and once timed (HIP events on the null stream), on
// `blocks` workgroups of kRateBlock threads.  For the ALU probes `out` is a
// device buffer of blocks * kRateBlock floats that receives each lane's
// chain values (so that no chain is dead code); for the stream probes `out`
// holds the source and destination, 2 * iters float4 elements each way
// (iters is then the element count per direction).  Returns 0, or a HIP
// error code.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kRateBlock = 256;
constexpr int kChains = 8;

enum Kind {
    K_FMA = 0,      // v_fma_f32 / v_fmac_f32
    K_MUL = 1,      // v_mul_f32
    K_RSQ = 2,      // v_rsq_f32
    K_ADD64 = 3,    // v_add_f64
    K_ACC64 = 4,    // v_fma_f32 + v_cvt_f64_f32 + v_add_f64 (the FP64 sum of an FP32 term)
    K_COPY = 5,     // float4 stream copy: reads and writes `iters` float4 each
    K_READ = 6,     // float4 stream read (one float per thread written)
};

__global__ __launch_bounds__(kRateBlock) void k_alu(int kind, int iters, float b, float c,
                                                    float *out) {
    const int t = blockIdx.x * kRateBlock + threadIdx.x;
    float a[kChains];
    double d[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
        a[k] = 1.0f + 1e-3f * (float)((t + k) & 255);
        d[k] = (double)a[k];
    }
    if (kind == K_FMA) {
#pragma unroll 4
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int k = 0; k < kChains; ++k) a[k] = fmaf(a[k], b, c);
    } else if (kind == K_MUL) {
#pragma unroll 4
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int k = 0; k < kChains; ++k) a[k] = a[k] * b;
    } else if (kind == K_RSQ) {
#pragma unroll 4
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int k = 0; k < kChains; ++k) a[k] = __builtin_amdgcn_rsqf(a[k]);
    } else if (kind == K_ADD64) {
        const double e = (double)c;
#pragma unroll 4
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int k = 0; k < kChains; ++k) d[k] = d[k] + e;
    } else {  // K_ACC64
#pragma unroll 4
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int k = 0; k < kChains; ++k) {
                a[k] = fmaf(a[k], b, c);
                d[k] = d[k] + (double)a[k];
            }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += a[k] + (float)d[k];
    out[t] = s;
}

__global__ __launch_bounds__(kRateBlock) void k_copy(const float4 *__restrict__ src,
                                                     float4 *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kRateBlock;
    for (int64_t i = (int64_t)blockIdx.x * kRateBlock + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

__global__ __launch_bounds__(kRateBlock) void k_read(const float4 *__restrict__ src, float *out,
                                                     int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kRateBlock;
    float s = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * kRateBlock + threadIdx.x; i < n; i += stride) {
        const float4 v = src[i];
        s += (v.x + v.y) + (v.z + v.w);
    }
    out[(int64_t)blockIdx.x * kRateBlock + threadIdx.x] = s;
}

hipError_t launch(int kind, int blocks, int iters, float *out) {
    if (kind <= K_ACC64) {
        k_alu<<<blocks, kRateBlock>>>(kind, iters, 0.999f, 1e-3f, out);
    } else if (kind == K_COPY) {
        float4 *buf = (float4 *)out;
        k_copy<<<blocks, kRateBlock>>>(buf, buf + iters, iters);
    } else {
        // the per-thread sums go after the source
        float4 *buf = (float4 *)out;
        k_read<<<blocks, kRateBlock>>>(buf, (float *)(buf + iters), iters);
    }
    return hipGetLastError();
}

}  // namespace

extern "C" int wnnc_rates_block(void) { return kRateBlock; }
extern "C" int wnnc_rates_chains(void) { return kChains; }

extern "C" int wnnc_rates_run(int kind, int blocks, int iters, float *out, float *ms_out) {
    if (kind < K_FMA || kind > K_READ || blocks <= 0 || iters <= 0 || !out || !ms_out)
        return (int)hipErrorInvalidValue;
    hipError_t e = launch(kind, blocks, iters, out);  // untimed: code load, clocks up
    if (e != hipSuccess) return (int)e;
    hipEvent_t t0, t1;
    if ((e = hipEventCreate(&t0)) != hipSuccess) return (int)e;
    if ((e = hipEventCreate(&t1)) != hipSuccess) {
        (void)hipEventDestroy(t0);
        return (int)e;
    }
    (void)hipEventRecord(t0, 0);
    e = launch(kind, blocks, iters, out);
    (void)hipEventRecord(t1, 0);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms_out, t0, t1);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    return (int)e;
}
