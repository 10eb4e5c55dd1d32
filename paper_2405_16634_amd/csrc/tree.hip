// Normalization (Sec. 5.1.1) and the octree build (Sec. 4.5) on the device.
//
// The octree over [-1,1]^3 with maximum depth D is the tree of Morton-code
// prefixes: quantize each coordinate to 15 bits, interleave into a 45-bit
// key, sort, and a node at depth d is a maximal run of sorted keys sharing
// their top 3d bits whose parent run holds more than one point.  With sorted
// keys this is decided locally: point i starts nodes at the depths
// L+1 .. min(max(L,R)+1, D), where L and R are the numbers of leading octal
// digits it shares with its left and right neighbours.  Numbering the nodes
// point by point, shallow to deep, yields a depth-first pre-order in which
// the first child of a node is the next node and a subtree is a contiguous
// index range.
#include <float.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "common.h"
#include "internal.h"

namespace wnnc {

// ------------------------------------------------------------ normalize --
// Each cloud c (caller rows off[c] .. off[c+1]) is normalized on its own.

constexpr int kNormBlocksPerCloud = 32;

int64_t normalize_tmp_doubles(int64_t nclouds) {
    return nclouds * (kNormBlocksPerCloud * 6 + 4) + 8;
}

__device__ inline int cloud_of_row(const int64_t *off, int nclouds, int64_t i) {
    int lo = 0, hi = nclouds;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// grid (kNormBlocksPerCloud, nclouds): per-block extremes of one cloud
__global__ __launch_bounds__(256) void k_minmax(const float *__restrict__ P,
                                                const int64_t *__restrict__ off,
                                                double *__restrict__ part) {
    const int c = blockIdx.y;
    const int64_t lo_i = off[c], hi_i = off[c + 1];
    float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    for (int64_t i = lo_i + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi_i;
         i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float v = P[3 * i + k];
            lo[k] = fminf(lo[k], v);
            hi[k] = fmaxf(hi[k], v);
        }
    }
    __shared__ float s[6][256];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        s[k][threadIdx.x] = lo[k];
        s[3 + k][threadIdx.x] = hi[k];
    }
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < d) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                s[k][threadIdx.x] = fminf(s[k][threadIdx.x], s[k][threadIdx.x + d]);
                s[3 + k][threadIdx.x] = fmaxf(s[3 + k][threadIdx.x], s[3 + k][threadIdx.x + d]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6)
        part[((int64_t)c * kNormBlocksPerCloud + blockIdx.x) * 6 + threadIdx.x] = s[threadIdx.x][0];
}

// One thread per cloud: extremes -> centre and scale in FP64.
__global__ void k_norm_finalize(const double *__restrict__ part, int nclouds,
                                double *__restrict__ cs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nclouds) return;
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = DBL_MAX;
        hi[k] = -DBL_MAX;
    }
    for (int b = 0; b < kNormBlocksPerCloud; ++b)
        for (int k = 0; k < 3; ++k) {
            lo[k] = fmin(lo[k], part[((int64_t)c * kNormBlocksPerCloud + b) * 6 + k]);
            hi[k] = fmax(hi[k], part[((int64_t)c * kNormBlocksPerCloud + b) * 6 + 3 + k]);
        }
    double half = 0.0;
    for (int k = 0; k < 3; ++k) {
        cs[4 * c + k] = (lo[k] + hi[k]) / 2.0;
        half = fmax(half, (hi[k] - lo[k]) / 2.0);
    }
    cs[4 * c + 3] = half > 0.0 ? (10.0 / 11.0) / half : 1.0;
}

__global__ __launch_bounds__(256) void k_norm_apply(const float *P, int64_t n3, float *Q,
                                                    const int64_t *__restrict__ off, int nclouds,
                                                    const double *__restrict__ cs) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    const int k = (int)(i % 3);
    const int c = nclouds == 1 ? 0 : cloud_of_row(off, nclouds, i / 3);
    Q[i] = (float)(((double)P[i] - cs[4 * c + k]) * cs[4 * c + 3]);
}

// tmp layout: [partials | centre/scale (4 per cloud)]; returns the offset of
// the centre/scale block in tmp.
int64_t launch_normalize(const float *P, int64_t n, const int64_t *d_off, int nclouds,
                         float *P_norm, double *tmp, hipStream_t st) {
    double *cs = tmp + (int64_t)nclouds * kNormBlocksPerCloud * 6;
    hipLaunchKernelGGL(k_minmax, dim3(kNormBlocksPerCloud, nclouds), dim3(256), 0, st, P, d_off, tmp);
    hipLaunchKernelGGL(k_norm_finalize, dim3((nclouds + 63) / 64), dim3(64), 0, st, tmp, nclouds, cs);
    const int64_t n3 = 3 * n;
    hipLaunchKernelGGL(k_norm_apply, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, P, n3,
                       P_norm, d_off, nclouds, cs);
    return (int64_t)nclouds * kNormBlocksPerCloud * 6;
}

// ----------------------------------------------------------------- morton --

// Spread the low 15 bits of v so that bit b lands on bit 3b.
__device__ inline unsigned long long spread3(unsigned v) {
    unsigned long long x = v & 0x7fffu;
    x = (x | (x << 16)) & 0x00000000ff0000ffull;
    x = (x | (x << 8)) & 0x000000f00f00f00full;
    x = (x | (x << 4)) & 0x00000c30c30c30c3ull;
    x = (x | (x << 2)) & 0x0000249249249249ull;
    return x;
}

// Cell index of coordinate v along one axis at depth 15:
// floor((v + 1) 2^14) clamped to [0, 2^15 - 1], evaluated as
// floor(v 2^14) + 2^14, which is exact in FP32 (the scaling is by a power of
// two).  A coordinate on a split plane goes to the upper cell.
__device__ inline unsigned quantize15(float v) {
    float f = floorf(v * 16384.0f) + 16384.0f;
    f = fminf(fmaxf(f, 0.0f), 32767.0f);
    return (unsigned)f;
}

__global__ __launch_bounds__(256) void k_morton(const float *__restrict__ P, int64_t n,
                                                const int64_t *__restrict__ off, int nclouds,
                                                unsigned long long *__restrict__ keys,
                                                uint32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned qx = quantize15(P[3 * i]), qy = quantize15(P[3 * i + 1]), qz = quantize15(P[3 * i + 2]);
    const unsigned long long c = nclouds == 1 ? 0ull : (unsigned long long)cloud_of_row(off, nclouds, i);
    keys[i] = (c << kMortonBits) | (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
    vals[i] = (uint32_t)i;
}

// Cloud index of every sorted point (clouds stay contiguous and in order).
__global__ __launch_bounds__(256) void k_point_cloud(const unsigned long long *__restrict__ keys,
                                                     int64_t n, int32_t *__restrict__ cloud) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) cloud[i] = (int32_t)(keys[i] >> kMortonBits);
}

// ------------------------------------------------------------ radix sort --
// Stable LSD radix sort of (45-bit key, uint32 value), 8 bits per pass.

constexpr int kRsThreads = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kRsThreads * kRsItems;

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const unsigned long long *__restrict__ keys,
                                                        int64_t n, int shift,
                                                        uint32_t *__restrict__ hist, int ntiles) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
        int64_t i = base + k * kRsThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(unsigned)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(
    const unsigned long long *__restrict__ kin, const uint32_t *__restrict__ vin,
    unsigned long long *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n, int shift,
    const uint32_t *__restrict__ offs, int ntiles) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[kRsThreads / kWave][256];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    const unsigned long long lt = (1ull << lane) - 1ull;
    run[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsItems; ++r) {
#pragma unroll
        for (int w = 0; w < kRsThreads / kWave; ++w) wc[w][tid] = 0;
        __syncthreads();
        const int64_t i = base + r * kRsThreads + tid;
        const bool valid = i < n;
        unsigned long long key = valid ? kin[i] : 0ull;
        uint32_t val = valid ? vin[i] : 0u;
        const unsigned dig = (unsigned)(key >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dig >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const unsigned rank = (unsigned)__popcll(peers & lt);
        if (valid && rank == 0) wc[wv][dig] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            uint32_t c[kRsThreads / kWave];
#pragma unroll
            for (int w = 0; w < kRsThreads / kWave; ++w) c[w] = wc[w][tid];
            uint32_t b = run[tid];
#pragma unroll
            for (int w = 0; w < kRsThreads / kWave; ++w) {
                wc[w][tid] = b;
                b += c[w];
            }
            run[tid] = b;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wc[wv][dig] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- nodes --

// Number of leading octal digits (of 15) shared by two keys; -1 for keys of
// different clouds.
__device__ inline int lcp_digits(unsigned long long a, unsigned long long b) {
    unsigned long long x = a ^ b;
    if (x == 0ull) return 15;
    if (x >> kMortonBits) return -1;
    return (__clzll(x) - (64 - kMortonBits)) / 3;
}

__device__ inline void neighbour_lcp(const unsigned long long *keys, int64_t n, int64_t i, int D,
                                     int *L, int *R) {
    const unsigned long long k = keys[i];
    int l = i > 0 ? lcp_digits(keys[i - 1], k) : -1;
    int r = i + 1 < n ? lcp_digits(k, keys[i + 1]) : -1;
    *L = l > D ? D : l;
    *R = r > D ? D : r;
}

// First sorted position after i whose key leaves the depth-d cell of key i
// (at depth 0 the cell is the cloud: the shift keeps only the cloud bits).
__device__ inline int64_t run_end(const unsigned long long *keys, int64_t n, int64_t i, int d) {
    const int shift = 3 * (15 - d);
    const unsigned long long pre = keys[i] >> shift;
    int64_t lo = i, step = 1;
    while (lo + step < n && (keys[lo + step] >> shift) == pre) {
        lo += step;
        step <<= 1;
    }
    int64_t hi = lo + step < n ? lo + step : n;  // keys[hi] differs, or hi == n
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        if ((keys[mid] >> shift) == pre)
            lo = mid;
        else
            hi = mid;
    }
    return hi;
}

// First sorted position of the run of depth-d cells that holds i (the
// mirror of run_end).
__device__ inline int64_t run_start(const unsigned long long *keys, int64_t i, int d) {
    const int shift = 3 * (15 - d);
    const unsigned long long pre = keys[i] >> shift;
    int64_t hi = i, step = 1;
    while (hi - step >= 0 && (keys[hi - step] >> shift) == pre) {
        hi -= step;
        step <<= 1;
    }
    int64_t lo = hi - step >= 0 ? hi - step : -1;  // keys[lo] differs, or lo == -1
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        if ((keys[mid] >> shift) == pre)
            hi = mid;
        else
            lo = mid;
    }
    return hi;
}

// The nodes whose first point is i, outermost first (pre-order), as
// emit(depth, end, leaf).  A node at depth d >= 1 is there when its parent
// (the depth d-1 run holding i) holds more than K points; it is a leaf when
// it holds at most K points or d == D.  With K = 1 (Alg. 4's tree) these
// are the depths from one below the common prefix with the left neighbour
// down to where i is alone, with no search.  Returns the node count.
template <class Emit>
__device__ inline int node_chain(const unsigned long long *keys, int64_t n, int64_t i, int D,
                                 int K, Emit &&emit) {
    int L, R;
    neighbour_lcp(keys, n, i, D, &L, &R);
    if (L >= D) return 0;
    if (K <= 1) {
        int hi = (L > R ? L : R) + 1;
        if (hi > D) hi = D;
        for (int d = L + 1; d <= hi; ++d) {
            const int64_t end = run_end(keys, n, i, d);
            emit(d, end, (end - i == 1) || (d == D));
        }
        return hi - L;
    }
    int cnt = 0;
    for (int d = L + 1; d <= D; ++d) {
        if (d >= 1) {
            const int64_t pb = d - 1 == L ? run_start(keys, i, L) : i;
            if (run_end(keys, n, i, d - 1) - pb <= K) break;
        }
        const int64_t end = run_end(keys, n, i, d);
        const bool leaf = end - i <= K || d == D;
        emit(d, end, leaf);
        ++cnt;
        if (leaf) break;
    }
    return cnt;
}

__global__ __launch_bounds__(256) void k_count_nodes(const unsigned long long *__restrict__ keys,
                                                     int64_t n, int D, int K,
                                                     uint32_t *__restrict__ counts) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        counts[n] = 0;
        return;
    }
    if (K <= 1) {  // no run boundaries needed for the count
        int L, R;
        neighbour_lcp(keys, n, i, D, &L, &R);
        int hi = (L > R ? L : R) + 1;
        if (hi > D) hi = D;
        counts[i] = L >= D ? 0u : (uint32_t)(hi - L);
        return;
    }
    counts[i] = (uint32_t)node_chain(keys, n, i, D, K, [](int, int64_t, bool) {});
}

__global__ __launch_bounds__(256) void k_emit_nodes(const unsigned long long *__restrict__ keys,
                                                    int64_t n, int D, int K,
                                                    const uint32_t *__restrict__ node_off,
                                                    int4 *__restrict__ topo,
                                                    uint32_t *__restrict__ strad_flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t idx = node_off[i];
    node_chain(keys, n, i, D, K, [&](int d, int64_t end, bool leaf) {
        topo[idx] = make_int4((int)node_off[end], (int)i, (int)end, d | ((leaf ? 1 : 0) << 4));
        strad_flag[idx] = ((i / kChunk) != ((end - 1) / kChunk)) ? 1u : 0u;
        ++idx;
    });
}

__global__ __launch_bounds__(256) void k_gather_roots(const uint32_t *__restrict__ node_off,
                                                      const int64_t *__restrict__ off, int nclouds,
                                                      int32_t *__restrict__ roots) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c <= nclouds) roots[c] = (int32_t)node_off[off[c]];
}

// Extract every third bit (bit 3b of x -> bit b), 15 bits.
__device__ inline unsigned compact3_15(unsigned long long x) {
    x &= 0x1249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x7fffull;
    return (unsigned)x;
}

// Static parts of the node records: the point range of every record (the
// moment passes write the rest), and the geometry of every node for
// searches by distance (the neighbour search): a single-point leaf holds its
// point (x, y, z, -1); any other node its cell (lower corner x, y, z, side),
// from the Morton key of its first point.
__global__ __launch_bounds__(256) void k_node_cells(const int4 *__restrict__ topo,
                                                    const unsigned long long *__restrict__ keys,
                                                    const float4 *__restrict__ pts, int64_t m,
                                                    float4 *__restrict__ cells,
                                                    float4 *__restrict__ mom) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int4 t = topo[k];
    // the parts of the record that no moment pass writes: flags,
    // skip pointer, point range; of a single-point leaf, whose representative
    // is its point whatever its attribute, also its position (hi = the
    // point, lo = 0) and threshold (-1: every target takes it)
    const bool single = (t.w & kRecLeaf) && t.z - t.y == 1;
    float4 r0 = make_float4(0.f, 0.f, 0.f, __int_as_float(t.w & 31));
    float4 r2 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (single) {
        const float4 q = pts[t.y];
        r0 = make_float4(q.x, q.y, q.z, __int_as_float((t.w & 31) | kRecSingle));
        r2.w = -1.0f;
    }
    const float4 r1 = make_float4(0.f, 0.f, 0.f, __int_as_float(t.x));
    const float4 r3 = make_float4(__int_as_float(t.y), __int_as_float(t.z), 0.f, 0.f);
    float4 *ra = mom + kRecStride * k;
    ra[0] = r0, ra[1] = r1, ra[2] = r2, ra[3] = r3;
    if (single) {
        cells[k] = make_float4(r0.x, r0.y, r0.z, -1.0f);
        return;
    }
    const int depth = t.w & 15;
    const int sh = kMaxDepth - depth;
    const float w = ldexpf(1.0f, 1 - depth);
    const unsigned long long mk = keys[t.y] & ((1ull << kMortonBits) - 1ull);
    cells[k] = make_float4(-1.0f + (float)(compact3_15(mk >> 2) >> sh) * w,
                           -1.0f + (float)(compact3_15(mk >> 1) >> sh) * w,
                           -1.0f + (float)(compact3_15(mk) >> sh) * w, w);
}

__global__ __launch_bounds__(256) void k_gather_points(const float *__restrict__ P,
                                                       const uint32_t *__restrict__ perm,
                                                       int64_t n, float4 *__restrict__ pts) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = perm[i];
    pts[i] = make_float4(P[3 * (int64_t)j], P[3 * (int64_t)j + 1], P[3 * (int64_t)j + 2], 0.0f);
}

// Straddlers (nodes whose points cross a chunk boundary of the moment pass)
// are numbered wide ones first: a wide straddler has more chunks in between
// than a wavefront has lanes and is summed by a whole workgroup, the others
// by a wavefront each.  On entry flag marks the straddlers; on return flag
// marks the narrow ones and wflag the wide ones (both m + 1 entries, the
// last 0, for the exclusive scans that number them).
__global__ __launch_bounds__(256) void k_split_wide(const int4 *__restrict__ topo, int64_t m,
                                                    uint32_t *__restrict__ flag,
                                                    uint32_t *__restrict__ wflag) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m || !flag[k]) return;
    const int4 t = topo[k];
    const bool wide = (t.z - 1) / kChunk - t.y / kChunk - 1 > kWave;
    flag[k] = wide ? 0u : 1u;
    wflag[k] = wide ? 1u : 0u;
}

// Slot of every straddler (wide ones 0 .. n_wide - 1, then the narrow ones)
// and the moment pass's view of every node.
__global__ __launch_bounds__(256) void k_strad_compact(const uint32_t *__restrict__ flag,
                                                       const uint32_t *__restrict__ slot,
                                                       const uint32_t *__restrict__ wflag,
                                                       const uint32_t *__restrict__ wslot,
                                                       const int4 *__restrict__ topo, int64_t m,
                                                       int32_t *__restrict__ node_strad,
                                                       int32_t *__restrict__ strad_node,
                                                       int4 *__restrict__ strad_topo,
                                                       int2 *__restrict__ mnode) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int4 t = topo[k];
    const int n_wide = (int)wslot[m];
    const int sl = wflag[k] ? (int)wslot[k] : (flag[k] ? n_wide + (int)slot[k] : -1);
    node_strad[k] = sl;
    if (sl >= 0) {
        strad_node[sl] = (int32_t)k;
        strad_topo[sl] = t;
        mnode[k] = make_int2(t.y, -1 - sl);
    } else {
        mnode[k] = make_int2(t.y, t.z | (topo_depth(t.w) << kMnodeEndBits));
    }
}

__global__ __launch_bounds__(256) void k_tail_count(const int32_t *__restrict__ strad_node,
                                                    const int4 *__restrict__ topo, int ns,
                                                    uint32_t *__restrict__ cnt) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    const int e = topo[strad_node[s]].z;
    atomicAdd(&cnt[(e - 1) / kChunk], 1u);
}

// (straddler slot, end point) of every straddler, listed under the chunk
// its range ends in
__global__ __launch_bounds__(256) void k_tail_fill(const int32_t *__restrict__ strad_node,
                                                   const int4 *__restrict__ topo, int ns,
                                                   uint32_t *__restrict__ cursor,
                                                   int2 *__restrict__ list) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    const int e = topo[strad_node[s]].z;
    const uint32_t q = atomicAdd(&cursor[(e - 1) / kChunk], 1u);
    list[q] = make_int2(s, e);
}

// ------------------------------------------------------------------- host --

static inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Builds the forest over the normalized points P (caller order); the cloud
// ranges are ctx->offsets (host) / ctx->d_offsets (device, already copied).
// Morton keys of the n caller-order points P (cloud index above the 45
// Morton bits when nclouds > 1) and a stable LSD sort, 8 bits per pass: on
// return ka holds the sorted keys and va the caller index of each.  An odd
// pass count leaves the result in the second buffer pair, which then becomes
// the first.  Uses ctx->hist and ctx->scan_tmp (sized here for n).
hipError_t morton_sort(wnnc_ctx_s *ctx, const float *P, int64_t n, int nclouds, int passes,
                       DevBuf<unsigned long long> &ka, DevBuf<unsigned long long> &kb,
                       DevBuf<uint32_t> &va, DevBuf<uint32_t> &vb) {
    hipStream_t st = ctx->stream;
    const int ntiles = (int)((n + kRsTile - 1) / kRsTile);
    const int64_t hsize = (int64_t)256 * ntiles;
    TRY(ka.ensure(n));
    TRY(kb.ensure(n));
    TRY(va.ensure(n));
    TRY(vb.ensure(n));
    TRY(ctx->hist.ensure(hsize));
    TRY(ctx->scan_tmp.ensure(scan_tmp_size(16 * (hsize > n + 1 ? hsize : n + 1) + 16)));
    hipLaunchKernelGGL(k_morton, dim3(blocks_for(n, 256)), dim3(256), 0, st, P, n,
                       ctx->d_offsets.p, nclouds, ka.p, va.p);
    unsigned long long *kin = ka.p, *kout = kb.p;
    uint32_t *vin = va.p, *vout = vb.p;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_rs_hist, dim3(ntiles), dim3(kRsThreads), 0, st, kin, n, shift,
                           ctx->hist.p, ntiles);
        TRY(exclusive_scan_u32(ctx->hist.p, ctx->hist.p, hsize, ctx->scan_tmp.p, st));
        hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(kRsThreads), 0, st, kin, vin, kout,
                           vout, n, shift, ctx->hist.p, ntiles);
        unsigned long long *tk = kin;
        kin = kout;
        kout = tk;
        uint32_t *tv = vin;
        vin = vout;
        vout = tv;
    }
    if (passes & 1) {
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    return hipGetLastError();
}

hipError_t build_tree(wnnc_ctx_s *ctx, const float *P) {
    const int64_t n = ctx->n;
    const int D = ctx->depth;
    const int nclouds = ctx->nclouds;
    hipStream_t st = ctx->stream;
    const int64_t nchunks = (n + kChunk - 1) / kChunk;
    const int ntiles = (int)((n + kRsTile - 1) / kRsTile);
    const int64_t hsize = (int64_t)256 * ntiles;
    int cloud_bits = 0;
    while ((1ll << cloud_bits) < nclouds) ++cloud_bits;
    const int passes = (kMortonBits + cloud_bits + 7) / 8;

    TRY(ctx->pts.ensure(n));
    TRY(ctx->perm.ensure(n));
    TRY(ctx->node_off.ensure(n + 1));
    TRY(ctx->keys_a.ensure(n));
    TRY(ctx->keys_b.ensure(n));
    TRY(ctx->vals_b.ensure(n));
    TRY(ctx->u32_tmp.ensure(n + 1));
    TRY(ctx->hist.ensure(hsize));
    TRY(ctx->tail_off.ensure(nchunks + 1));
    TRY(ctx->chunk_tot.ensure((int64_t)kMomSlots * nchunks));
    TRY(ctx->cloud_of.ensure(n));
    TRY(ctx->va.ensure(n));
    TRY(ctx->vb.ensure(n));
    TRY(ctx->vr.ensure(n));
    TRY(ctx->rho.ensure(n));
    TRY(ctx->scalars.ensure(nclouds));
    TRY(ctx->pair_ctr.ensure(kOpKinds));
    TRY(ctx->finite_flag.ensure(1));
    {
        int64_t big = hsize > n + 1 ? hsize : n + 1;
        TRY(ctx->scan_tmp.ensure(scan_tmp_size(16 * big + 16)));
    }

    TRY(morton_sort(ctx, P, n, nclouds, passes, ctx->keys_a, ctx->keys_b, ctx->perm,
                    ctx->vals_b));
    hipLaunchKernelGGL(k_point_cloud, dim3(blocks_for(n, 256)), dim3(256), 0, st, ctx->keys_a.p, n,
                       ctx->cloud_of.p);

    // nodes started per point -> pre-order offsets; M is read back once
    hipLaunchKernelGGL(k_count_nodes, dim3(blocks_for(n + 1, 256)), dim3(256), 0, st,
                       ctx->keys_a.p, n, D, ctx->leaf_cap, ctx->u32_tmp.p);
    TRY(exclusive_scan_u32(ctx->u32_tmp.p, ctx->node_off.p, n + 1, ctx->scan_tmp.p, st));
    // first node of every cloud (node_off at the cloud starts); the last
    // entry is M
    TRY(ctx->d_roots.ensure(nclouds + 1));
    hipLaunchKernelGGL(k_gather_roots, dim3((nclouds + 256) / 256), dim3(256), 0, st,
                       ctx->node_off.p, ctx->d_offsets.p, nclouds, ctx->d_roots.p);
    ctx->roots.resize(nclouds + 1);
    TRY(hipMemcpyAsync(ctx->roots.data(), ctx->d_roots.p, (size_t)(nclouds + 1) * sizeof(int32_t),
                       hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    const int64_t m = ctx->roots[nclouds];
    if (m > kMaxNodes) return hipErrorNotSupported;  // beyond 32-bit record offsets
    ctx->m = m;

    TRY(ctx->topo.ensure(m));
    TRY(ctx->node_strad.ensure(m));
    TRY(ctx->mom.ensure(kRecStride * m));
    TRY(ctx->mnode.ensure(m));
    TRY(ctx->mflag.ensure(m + 1));
    TRY(ctx->mslot.ensure(m + 1));

    TRY(hipMemsetAsync(ctx->mflag.p, 0, (size_t)(m + 1) * sizeof(uint32_t), st));
    hipLaunchKernelGGL(k_emit_nodes, dim3(blocks_for(n, 256)), dim3(256), 0, st, ctx->keys_a.p,
                       n, D, ctx->leaf_cap, ctx->node_off.p, ctx->topo.p, ctx->mflag.p);
    hipLaunchKernelGGL(k_gather_points, dim3(blocks_for(n, 256)), dim3(256), 0, st, P,
                       ctx->perm.p, n, ctx->pts.p);
    TRY(ctx->cells.ensure(m));
    hipLaunchKernelGGL(k_node_cells, dim3(blocks_for(m, 256)), dim3(256), 0, st, ctx->topo.p,
                       ctx->keys_a.p, ctx->pts.p, m, ctx->cells.p, ctx->mom.p);
    TRY(ctx->wflag.ensure(m + 1));
    TRY(ctx->wslot.ensure(m + 1));
    TRY(hipMemsetAsync(ctx->wflag.p, 0, (size_t)(m + 1) * sizeof(uint32_t), st));
    hipLaunchKernelGGL(k_split_wide, dim3(blocks_for(m, 256)), dim3(256), 0, st, ctx->topo.p, m,
                       ctx->mflag.p, ctx->wflag.p);
    TRY(exclusive_scan_u32(ctx->mflag.p, ctx->mslot.p, m + 1, ctx->scan_tmp.p, st));
    TRY(exclusive_scan_u32(ctx->wflag.p, ctx->wslot.p, m + 1, ctx->scan_tmp.p, st));
    uint32_t nn32 = 0, nw32 = 0;
    TRY(hipMemcpyAsync(&nn32, ctx->mslot.p + m, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(&nw32, ctx->wslot.p + m, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    const int64_t ns = (int64_t)nn32 + nw32;
    ctx->n_strad = (int32_t)ns;
    ctx->n_wide = (int32_t)nw32;
    TRY(ctx->strad_node.ensure(ns + 1));
    TRY(ctx->strad_topo.ensure(ns + 1));
    TRY(ctx->tail_list.ensure(ns + 1));
    TRY(ctx->head.ensure((int64_t)kMomSlots * (ns + 1)));
    TRY(ctx->tail.ensure((int64_t)kMomSlots * (ns + 1)));
    hipLaunchKernelGGL(k_strad_compact, dim3(blocks_for(m, 256)), dim3(256), 0, st, ctx->mflag.p,
                       ctx->mslot.p, ctx->wflag.p, ctx->wslot.p, ctx->topo.p, m,
                       ctx->node_strad.p, ctx->strad_node.p, ctx->strad_topo.p, ctx->mnode.p);
    // chunk -> straddlers whose range ends inside it (CSR); counts reuse mflag
    uint32_t *tcnt = ctx->u32_tmp.p;  // n+1 >= chunks+1 entries
    TRY(hipMemsetAsync(tcnt, 0, (size_t)(nchunks + 1) * sizeof(uint32_t), st));
    if (ns > 0)
        hipLaunchKernelGGL(k_tail_count, dim3(blocks_for(ns, 256)), dim3(256), 0, st,
                           ctx->strad_node.p, ctx->topo.p, (int)ns, tcnt);
    TRY(exclusive_scan_u32(tcnt, ctx->tail_off.p, nchunks + 1, ctx->scan_tmp.p, st));
    uint32_t *cursor = ctx->mslot.p;  // free again: m+1 >= chunks+1 entries
    TRY(hipMemcpyAsync(cursor, ctx->tail_off.p, (size_t)(nchunks + 1) * sizeof(uint32_t),
                       hipMemcpyDeviceToDevice, st));
    if (ns > 0)
        hipLaunchKernelGGL(k_tail_fill, dim3(blocks_for(ns, 256)), dim3(256), 0, st,
                           ctx->strad_node.p, ctx->topo.p, (int)ns, cursor, ctx->tail_list.p);
    TRY(hipStreamSynchronize(st));
    TRY(hipMemsetAsync(ctx->pair_ctr.p, 0, kOpKinds * sizeof(unsigned long long), st));
    return hipGetLastError();
}

// The ancestors of each task's first node, from its cloud's root down: the
// nodes at which a part of a split walk re-evaluates its lanes' decisions
// (none for a walk that starts at the root).  At most one ancestor per
// depth and 8 children per node are examined, so the loops end.
__global__ __launch_bounds__(256) void k_task_chains(const int4 *__restrict__ tasks,
                                                     const int32_t *__restrict__ cloud,
                                                     const int32_t *__restrict__ roots,
                                                     const int4 *__restrict__ topo, int ntasks,
                                                     int32_t *__restrict__ chain) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntasks) return;
    const int4 tk = tasks[t];
    const int nbeg = tk.z;
    int node = roots[cloud[tk.x]];
    int32_t *out = chain + (int64_t)t * kChainStride;
    int cnt = 0;
    for (int d = 0; d < kMaxDepth && node < nbeg; ++d) {
        out[1 + cnt++] = node;
        int ch = node + 1;  // the child whose subtree holds the first node
        for (int c = 0; c < 8; ++c) {
            const int sk = topo[ch].x;
            if (sk > nbeg) break;
            ch = sk;
        }
        node = ch;
    }
    out[0] = cnt;
}

// Wavefront tasks for tile shape tpl: each cloud's sorted targets cut into
// runs of 64 * tpl, in Morton order, cloud after cloud.  The partial-sum
// slot of a task is its index, so a cloud's slots are contiguous.
hipError_t make_tasks(wnnc_ctx_s *ctx, int tpl, int split) {
    const int per = kWave * tpl;
    const bool use_plan = split > 0 && tpl == 1 && !ctx->plan.empty();
    std::vector<int4> tk, sg;
    std::vector<int32_t> slot, sslot;
    std::vector<int32_t> lo(ctx->nclouds + 1);
    std::vector<int32_t> cut;
    int32_t g = 0, nparts = 0;
    for (int c = 0; c < ctx->nclouds; ++c) {
        lo[c] = g;
        const int64_t a = ctx->offsets[c], b = ctx->offsets[c + 1];
        const int root = ctx->roots[c], rend = ctx->roots[c + 1];
        for (int64_t f = a; f < b; f += per, ++g) {
            const int l = (int)(f + per < b ? f + per : b);
            // cut points: nodes the recorded walk reaches near every
            // split-th visit (the walk moves forward in pre-order, so they
            // increase)
            cut.clear();
            if (use_plan) {
                const int32_t *pl = ctx->plan.data() + (size_t)g * kPlanStride;
                const int64_t V = pl[0];
                const int P = (int)((V + split - 1) / split);
                const int kmax = (int)std::min<int64_t>(kPlanCap, V > 0 ? (V - 1) / kPlanStep : 0);
                int prev = root;
                for (int q = 1; q < P; ++q) {
                    const int64_t v = V * q / P;
                    int k = (int)((v + kPlanStep / 2) / kPlanStep);
                    k = std::min(std::max(k, 1), kmax);
                    if (k < 1) continue;
                    const int nd = pl[k];
                    if (nd > prev && nd < rend) {
                        cut.push_back(nd);
                        prev = nd;
                    }
                }
            }
            if (cut.empty()) {
                tk.push_back(make_int4((int)f, l, root, rend));
                slot.push_back(g);
                continue;
            }
            const int P = (int)cut.size() + 1;
            sg.push_back(make_int4((int)f, l, nparts, nparts + P));
            sslot.push_back(g);
            int s0 = root;
            for (int q = 0; q < P; ++q) {
                const int e = q + 1 < P ? cut[q] : rend;
                tk.push_back(make_int4((int)f, l, s0, e));
                slot.push_back(-1 - (nparts + q));
                s0 = e;
            }
            nparts += P;
        }
    }
    lo[ctx->nclouds] = g;
    const int64_t nt = (int64_t)tk.size(), ns = (int64_t)sg.size();
    // per group, its part range, when the groups are the 64-point blocks of
    // the sorted points (one group per wavefront, every cloud starting at a
    // multiple of 64): a moment pass can then combine the parts itself
    bool aligned = tpl == 1 && ns > 0;
    for (int c = 0; c < ctx->nclouds && aligned; ++c) aligned = ctx->offsets[c] % kWave == 0;
    ctx->gtab_ok = false;
    if (aligned) {
        std::vector<int2> gt((size_t)g, make_int2(0, 0));
        for (int64_t q = 0; q < ns; ++q) gt[(size_t)sslot[q]] = make_int2(sg[q].z, sg[q].w);
        TRY(ctx->gtab.ensure(g));
        TRY(hipMemcpyAsync(ctx->gtab.p, gt.data(), (size_t)g * sizeof(int2), hipMemcpyHostToDevice,
                           ctx->stream));
        TRY(hipStreamSynchronize(ctx->stream));  // (gt is released on return)
        ctx->gtab_ok = true;
    }
    TRY(ctx->tasks.ensure(nt));
    TRY(ctx->task_slot.ensure(nt));
    TRY(ctx->task_lo.ensure(ctx->nclouds + 1));
    TRY(ctx->partial.ensure(3 * (int64_t)g));
    TRY(ctx->split_groups.ensure(ns > 0 ? ns : 1));
    TRY(ctx->split_slot.ensure(ns > 0 ? ns : 1));
    TRY(ctx->parts.ensure(nparts > 0 ? (int64_t)nparts * 3 * kWave : 1));
    TRY(hipMemcpyAsync(ctx->tasks.p, tk.data(), (size_t)nt * sizeof(int4), hipMemcpyHostToDevice,
                       ctx->stream));
    TRY(hipMemcpyAsync(ctx->task_slot.p, slot.data(), (size_t)nt * sizeof(int32_t),
                       hipMemcpyHostToDevice, ctx->stream));
    TRY(hipMemcpyAsync(ctx->task_lo.p, lo.data(), lo.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, ctx->stream));
    if (ns > 0) {
        TRY(hipMemcpyAsync(ctx->split_groups.p, sg.data(), (size_t)ns * sizeof(int4),
                           hipMemcpyHostToDevice, ctx->stream));
        TRY(hipMemcpyAsync(ctx->split_slot.p, sslot.data(), (size_t)ns * sizeof(int32_t),
                           hipMemcpyHostToDevice, ctx->stream));
    }
    TRY(ctx->task_chain.ensure(nt * kChainStride));
    if (nt > 0)
        hipLaunchKernelGGL(k_task_chains, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0,
                           ctx->stream, ctx->tasks.p, ctx->cloud_of.p, ctx->d_roots.p,
                           ctx->topo.p, (int)nt, ctx->task_chain.p);
    TRY(hipGetLastError());
    // the host vectors are released on return: wait for the copies
    TRY(hipStreamSynchronize(ctx->stream));
    ctx->ntasks = (int)nt;
    ctx->ngroups = g;
    ctx->nparts = nparts;
    ctx->nsplit = (int)ns;
    ctx->tpl = tpl;
    ctx->split = split;
    return hipSuccess;
}

hipError_t sort_queries(wnnc_ctx_s *ctx, const float *Q, int64_t M) {
    TRY(morton_sort(ctx, Q, M, 1, (kMortonBits + 7) / 8, ctx->qkeys_a, ctx->qkeys_b, ctx->qperm,
                    ctx->qvals_b));
    TRY(ctx->qpts.ensure(M));
    hipLaunchKernelGGL(k_gather_points, dim3(blocks_for(M, 256)), dim3(256), 0, ctx->stream, Q,
                       ctx->qperm.p, M, ctx->qpts.p);
    return hipGetLastError();
}

}  // namespace wnnc
