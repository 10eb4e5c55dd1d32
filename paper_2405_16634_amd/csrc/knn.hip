// k = 16 nearest neighbours of every point within its cloud, on the octree,
// and the neighbourhood features of the learned warm start: the offsets to
// the 16 neighbours in increasing distance, divided by their RMS length.
//
// One lane per target.  The candidate list (squared distance, sorted index)
// lives in registers, sorted ascending; it is seeded with the target's
// Morton-order neighbours, which gives a tight radius from the start.  Each
// lane then walks its cloud's pre-order node range on its own, skipping a
// subtree whenever the box of its cell is farther than the current 16th
// candidate (cells come from the Morton key of the node's first point), and
// testing the points of the leaves it reaches.  Ties are broken by sorted
// index.  Requires points inside [-1,1]^3 (normalized clouds).
#include <float.h>

#include "common.h"
#include "internal.h"

namespace wnnc {

constexpr int kK = 16;

__device__ inline unsigned compact3(unsigned long long x) {
    x &= 0x1249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x7fffull;
    return (unsigned)x;
}

struct Cand {
    float d[kK];
    int j[kK];
};

__device__ inline bool better(float d, int j, float dd, int jj) {
    return d < dd || (d == dd && j < jj);
}

// insert (d, j) into the sorted list if it beats the last entry
__device__ inline void offer(Cand &c, float d, int j) {
    if (!better(d, j, c.d[kK - 1], c.j[kK - 1])) return;
    c.d[kK - 1] = d;
    c.j[kK - 1] = j;
#pragma unroll
    for (int k = kK - 1; k > 0; --k) {
        if (better(c.d[k], c.j[k], c.d[k - 1], c.j[k - 1])) {
            const float td = c.d[k];
            const int tj = c.j[k];
            c.d[k] = c.d[k - 1];
            c.j[k] = c.j[k - 1];
            c.d[k - 1] = td;
            c.j[k - 1] = tj;
        }
    }
}

// squared distance from p to the depth-d cell of key (FP32 box)
__device__ inline float cell_dist2(unsigned long long key, int d, float px, float py, float pz) {
    const int sh = kMaxDepth - d;
    const float w = ldexpf(1.0f, 1 - d);
    const unsigned long long mk = key & ((1ull << kMortonBits) - 1ull);
    const float lx = -1.0f + (float)(compact3(mk >> 2) >> sh) * w;
    const float ly = -1.0f + (float)(compact3(mk >> 1) >> sh) * w;
    const float lz = -1.0f + (float)(compact3(mk) >> sh) * w;
    const float dx = fmaxf(fmaxf(lx - px, px - (lx + w)), 0.0f);
    const float dy = fmaxf(fmaxf(ly - py, py - (ly + w)), 0.0f);
    const float dz = fmaxf(fmaxf(lz - pz, pz - (lz + w)), 0.0f);
    return dx * dx + dy * dy + dz * dz;
}

__global__ __launch_bounds__(256) void k_knn(const float4 *__restrict__ pts,
                                             const unsigned long long *__restrict__ keys,
                                             const int4 *__restrict__ topo,
                                             const int32_t *__restrict__ cloud,
                                             const int64_t *__restrict__ off,
                                             const int32_t *__restrict__ roots, int n,
                                             int32_t *__restrict__ nbr, float *__restrict__ nd2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int c = cloud[t];
    const int lo = (int)off[c], hi = (int)off[c + 1];
    const float4 p = pts[t];
    Cand cd;
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        cd.d[k] = FLT_MAX;
        cd.j[k] = -1;
    }
    // seed with Morton-order neighbours; the walk below skips them
    const int s_lo = max(lo, t - kK / 2 - 1), s_hi = min(hi - 1, t + kK / 2 + 1);
    for (int j = s_lo; j <= s_hi; ++j) {
        if (j == t) continue;
        const float4 q = pts[j];
        const float dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
        offer(cd, fmaf(dx, dx, fmaf(dy, dy, dz * dz)), j);
    }
    int node = roots[c];
    const int rend = roots[c + 1];
    while (node < rend) {
        const int4 tp = topo[node];
        const int depth = tp.w & 15;
        const float bd = cell_dist2(keys[tp.y], depth, p.x, p.y, p.z);
        if (bd > cd.d[kK - 1]) {
            node = tp.x;
            continue;
        }
        if (tp.w & kRecLeaf) {
            for (int j = tp.y; j < tp.z; ++j) {
                if (j >= s_lo && j <= s_hi) continue;  // seeded (or the target)
                const float4 q = pts[j];
                const float dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
                offer(cd, fmaf(dx, dx, fmaf(dy, dy, dz * dz)), j);
            }
            node = tp.x;
        } else {
            node = node + 1;
        }
    }
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        nbr[(int64_t)t * kK + k] = cd.j[k];
        nd2[(int64_t)t * kK + k] = cd.d[k];
    }
}

// Features of sorted point t, written at its caller row: offsets to the 16
// neighbours (nearest first) divided by their RMS length; missing neighbours
// (clouds of fewer than 17 points) and zero RMS give zeros.  Optionally the
// neighbours' caller indices.
__global__ __launch_bounds__(256) void k_features(const float4 *__restrict__ pts,
                                                  const uint32_t *__restrict__ perm,
                                                  const int32_t *__restrict__ nbr, int n,
                                                  float *__restrict__ feat,
                                                  int32_t *__restrict__ nbr_caller) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float4 p = pts[t];
    float o[3 * kK];
    double s2 = 0.0;
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        const int j = nbr[(int64_t)t * kK + k];
        float ox = 0.f, oy = 0.f, oz = 0.f;
        if (j >= 0) {
            const float4 q = pts[j];
            ox = q.x - p.x, oy = q.y - p.y, oz = q.z - p.z;
            s2 += (double)ox * ox + (double)oy * oy + (double)oz * oz;
            ++cnt;
        }
        o[3 * k] = ox, o[3 * k + 1] = oy, o[3 * k + 2] = oz;
    }
    const double rms = cnt > 0 ? sqrt(s2 / cnt) : 0.0;
    const float inv = rms > 0.0 ? (float)(1.0 / rms) : 0.0f;
    const int64_t row = perm[t];
#pragma unroll
    for (int k = 0; k < 3 * kK; ++k) feat[row * (3 * kK) + k] = o[k] * inv;
    if (nbr_caller) {
#pragma unroll
        for (int k = 0; k < kK; ++k) {
            const int j = nbr[(int64_t)t * kK + k];
            nbr_caller[row * kK + k] = j >= 0 ? (int32_t)perm[j] : -1;
        }
    }
}

hipError_t launch_knn_features(wnnc_ctx_s *ctx, float *feat, int32_t *nbr_caller) {
    const int n = (int)ctx->n;
    hipStream_t st = ctx->stream;
    hipError_t e = ctx->knn_idx.ensure((int64_t)n * kK);
    if (e != hipSuccess) return e;
    e = ctx->knn_d2.ensure((int64_t)n * kK);
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_knn, dim3(nb), dim3(256), 0, st, ctx->pts.p, ctx->keys_a.p, ctx->topo.p,
                       ctx->cloud_of.p, ctx->d_offsets.p, ctx->d_roots.p, n, ctx->knn_idx.p,
                       ctx->knn_d2.p);
    hipLaunchKernelGGL(k_features, dim3(nb), dim3(256), 0, st, ctx->pts.p, ctx->perm.p,
                       ctx->knn_idx.p, n, feat, nbr_caller);
    return hipGetLastError();
}

}  // namespace wnnc
