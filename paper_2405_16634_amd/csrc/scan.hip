// Exclusive prefix sums of uint32 arrays (used by the tree build).
#include "common.h"
#include "internal.h"

namespace wnnc {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Exclusive scan of one value per thread over a 256-thread block.  Returns the
// exclusive prefix; *total receives the block sum.
__device__ inline uint32_t block_exclusive_256(uint32_t v, uint32_t *total) {
    __shared__ uint32_t wsum[kScanThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t o = __shfl_up(inc, d, kWave);
        if (lane >= d) inc += o;
    }
    if (lane == kWave - 1) wsum[wv] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / kWave; ++k) {
        if (k < wv) base += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t *__restrict__ in,
                                                              int64_t n,
                                                              uint32_t *__restrict__ bsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k * kScanThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t tot;
    block_exclusive_256(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of nb block sums in one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_single(uint32_t *__restrict__ bsum, int64_t nb) {
    __shared__ uint32_t tsum[1024];
    const int64_t per = (nb + 1023) / 1024;
    const int64_t lo = threadIdx.x * per;
    const int64_t hi = lo + per < nb ? lo + per : nb;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += bsum[i];
    tsum[threadIdx.x] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        uint32_t o = threadIdx.x >= d ? tsum[threadIdx.x - d] : 0;
        __syncthreads();
        tsum[threadIdx.x] += o;
        __syncthreads();
    }
    uint32_t run = tsum[threadIdx.x] - s;
    for (int64_t i = lo; i < hi; ++i) {
        uint32_t v = bsum[i];
        bsum[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t *__restrict__ in,
                                                            uint32_t *__restrict__ out, int64_t n,
                                                            const uint32_t *__restrict__ bsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_256(s, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

int64_t scan_tmp_size(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

// out[i] = sum_{k<i} in[k] for i < n.  in may equal out.  tmp holds
// scan_tmp_size(n) entries.
hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp,
                              hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, tmp);
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, st, tmp, nb);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, out, n, tmp);
    return hipGetLastError();
}

}  // namespace wnnc
