// k = 16 nearest neighbours of every point within its cloud, on the octree,
// and the neighbourhood features of the learned warm start: the offsets to
// the 16 neighbours in increasing distance, divided by their RMS length.
//
// One wavefront per group of 64 Morton-consecutive points of one cloud, one
// point per lane.  Each lane keeps a candidate list (squared distance, sorted
// index) in registers, sorted ascending, seeded with its Morton-order
// neighbours on both sides (a tight radius from the start).  The wavefront then walks the
// cloud's pre-order node range as one scalar loop: a subtree is skipped when
// its cell (built with the tree) is farther than every lane's current 16th
// candidate; the points of the leaves reached are offered to every lane
// that needs them.  Ties are broken by sorted index,
// so the result does not depend on the order in which points are offered.
// Requires points inside [-1,1]^3 (normalized clouds).
#include <float.h>

#include "common.h"
#include "internal.h"

namespace wnnc {

constexpr int kK = 16;

struct Cand {
    float d[kK];
    int j[kK];
};

// (d, j) sorts before (dd, jj).  Bitwise operators: no short-circuit
// branches, so the callers compile to compares and selects.
__device__ inline bool better(float d, int j, float dd, int jj) {
    return (d < dd) | ((d == dd) & (j < jj));
}

// Inserts (d, j) into the sorted list where `take` holds and (d, j) beats
// the last entry: every entry the new one beats moves down one place.
// Branch-free (selects only), so the list stays in the same registers.
__device__ inline void offer(Cand &c, float d, int j, bool take = true) {
    take = take & better(d, j, c.d[kK - 1], c.j[kK - 1]);
#pragma unroll
    for (int k = kK - 1; k > 0; --k) {
        const bool shift = take & better(d, j, c.d[k - 1], c.j[k - 1]);
        // beats entry k but not entry k-1
        const bool put = take & !shift & better(d, j, c.d[k], c.j[k]);
        c.d[k] = shift ? c.d[k - 1] : (put ? d : c.d[k]);
        c.j[k] = shift ? c.j[k - 1] : (put ? j : c.j[k]);
    }
    const bool first = take & better(d, j, c.d[0], c.j[0]);
    c.d[0] = first ? d : c.d[0];
    c.j[0] = first ? j : c.j[0];
}

typedef int v4i_knn __attribute__((ext_vector_type(4)));
typedef float v4f_knn __attribute__((ext_vector_type(4)));

// Wave-uniform loads through the constant address space (scalar loads).
__device__ inline int4 knn_ld_i4(const int4 *p) {
    const v4i_knn v = *(const __attribute__((address_space(4))) v4i_knn *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ inline float4 knn_ld_f4(const float4 *p) {
    const v4f_knn v = *(const __attribute__((address_space(4))) v4f_knn *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
// groups: per wavefront (first, last point; first, end node of the cloud),
// the 64-point groups of every cloud.
__global__ __launch_bounds__(kWave) void k_knn(const float4 *__restrict__ pts,
                                               const float4 *__restrict__ cells,
                                               const int4 *__restrict__ topo,
                                               const int4 *__restrict__ groups,
                                               const int64_t *__restrict__ off,
                                               const int32_t *__restrict__ cloud, int ngroups,
                                               int32_t *__restrict__ nbr,
                                               float *__restrict__ nd2) {
    const int g = blockIdx.x;
    if (g >= ngroups) return;
    const int lane = threadIdx.x;
    const int4 G = knn_ld_i4(groups + g);
    const int c = *(const __attribute__((address_space(4))) int *)(cloud + G.x);
    const int lo = (int)off[c], hi = (int)off[c + 1];
    const int t = G.x + lane;
    const bool valid = t < G.y;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    if (valid) p = pts[t];
    Cand cd;
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        cd.d[k] = FLT_MAX;
        cd.j[k] = -1;
    }
    // seed with the kK Morton-order neighbours on each side (one side alone
    // fills the list, which bounds the radius also where the curve jumps);
    // the walk below skips them
    const int s_lo = max(lo, t - kK), s_hi = min(hi - 1, t + kK);
#pragma unroll 1
    for (int q = -kK; q <= kK; ++q) {
        const int j = t + q;
        const bool in = valid && q != 0 && j >= s_lo && j <= s_hi;
        float4 r = p;
        if (in) r = pts[j];
        const float dx = r.x - p.x, dy = r.y - p.y, dz = r.z - p.z;
        offer(cd, fmaf(dx, dx, fmaf(dy, dy, dz * dz)), j, in);
    }
    // One pruned walk over the pre-order range [nb, ne), skipping the
    // subtree [hole, hole_end) (hole = -1: none).
    auto walk = [&](int nb, int ne, int hole, int hole_end) {
        int node = nb;
        while (node < ne) {
            if (node == hole) {
                node = hole_end;
                continue;
            }
            // the node and its geometry: two independent scalar loads
            const int4 tp = knn_ld_i4(topo + node);
            const float4 cb = knn_ld_f4(cells + node);
            if (cb.w < 0.0f) {  // a single-point leaf: its point directly
                const int j = tp.y;
                const float dx = cb.x - p.x, dy = cb.y - p.y, dz = cb.z - p.z;
                const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const bool take = valid & ((j < s_lo) | (j > s_hi)) &
                                  better(d2, j, cd.d[kK - 1], cd.j[kK - 1]);
                if (__ballot(take)) offer(cd, d2, j, take);
                node = tp.x;
                continue;
            }
            // each lane's distance to the node's cell
            const float bx = fmaxf(fmaxf(cb.x - p.x, p.x - (cb.x + cb.w)), 0.0f);
            const float by = fmaxf(fmaxf(cb.y - p.y, p.y - (cb.y + cb.w)), 0.0f);
            const float bz = fmaxf(fmaxf(cb.z - p.z, p.z - (cb.z + cb.w)), 0.0f);
            const bool need = valid & (bx * bx + by * by + bz * bz <= cd.d[kK - 1]);
            if (__ballot(need) == 0ull) {
                node = tp.x;
                continue;
            }
            if (tp.w & kRecLeaf) {
#pragma unroll 1
                for (int j = tp.y; j < tp.z; ++j) {
                    const float4 r = knn_ld_f4(pts + j);
                    const float dx = r.x - p.x, dy = r.y - p.y, dz = r.z - p.z;
                    const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    // seeded (or the target itself) points were offered already
                    const bool take = need & ((j < s_lo) | (j > s_hi)) &
                                      better(d2, j, cd.d[kK - 1], cd.j[kK - 1]);
                    if (__ballot(take)) offer(cd, d2, j, take);
                }
                node = tp.x;
            } else {
                node = node + 1;
            }
        }
    };
    // Nearest first: the deepest node holding the whole group (its home),
    // whose points give every lane a tight radius, then the rest of the
    // cloud's tree with that radius.  At most one node per depth and 8
    // children per node are examined, so the search ends on any input.
    int home = G.z;
    for (int d = 0; d < kMaxDepth; ++d) {
        const int4 th = knn_ld_i4(topo + home);
        if (th.w & kRecLeaf) break;
        int ch = home + 1;
        for (int q = 0; q < 7; ++q) {  // the child whose point range holds `first`
            const int4 tc = knn_ld_i4(topo + ch);
            if (tc.z > G.x) break;
            ch = tc.x;
        }
        if (knn_ld_i4(topo + ch).z < G.y) break;  // it does not hold the whole group
        home = ch;
    }
    const int home_end = knn_ld_i4(topo + home).x;
    walk(home, home_end, -1, 0);
    walk(G.z, G.w, home, home_end);
    if (valid) {
#pragma unroll
        for (int k = 0; k < kK; ++k) {
            nbr[(int64_t)t * kK + k] = cd.j[k];
            nd2[(int64_t)t * kK + k] = cd.d[k];
        }
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

// Neighbour-search groups: runs of sorted points inside one octree cell of
// depth kKnnGroupDepth (so of one cloud), cut every 64 points.  A wavefront
// walks the union of its lanes' search balls; capping the cell keeps that
// union small where points are sparse (64 Morton-consecutive isolated
// points can span much of the cloud's box), at the price of partly filled
// wavefronts there.
constexpr int kKnnGroupDepth = 6;

__global__ __launch_bounds__(256) void k_knn_brk(const unsigned long long *__restrict__ keys,
                                                 int n, uint32_t *__restrict__ brk) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int sh = 3 * (kMaxDepth - kKnnGroupDepth);  // the cloud index sits above the key
    brk[i] = (i == 0 || (keys[i] >> sh) != (keys[i - 1] >> sh)) ? 1u : 0u;
}

// run starts: runs[r] = first point of run r (rx = exclusive scan of brk)
__global__ __launch_bounds__(256) void k_knn_runs(const uint32_t *__restrict__ brk,
                                                  const uint32_t *__restrict__ rx, int n,
                                                  uint32_t *__restrict__ runs) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n && brk[i]) runs[rx[i]] = (uint32_t)i;
}

// group starts: every 64th point of its run
__global__ __launch_bounds__(256) void k_knn_gflag(const uint32_t *__restrict__ brk,
                                                   const uint32_t *__restrict__ rx,
                                                   const uint32_t *__restrict__ runs, int n,
                                                   uint32_t *__restrict__ gs) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t r = rx[i] + brk[i] - 1u;
    gs[i] = ((i - (int)runs[r]) & (kWave - 1)) == 0 ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_knn_groups(const uint32_t *__restrict__ brk,
                                                    const uint32_t *__restrict__ rx,
                                                    const uint32_t *__restrict__ runs,
                                                    const uint32_t *__restrict__ gs,
                                                    const uint32_t *__restrict__ gx, int n,
                                                    const int32_t *__restrict__ cloud,
                                                    const int32_t *__restrict__ roots,
                                                    int4 *__restrict__ groups,
                                                    uint32_t *__restrict__ count) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if (i == n - 1) {
        count[0] = gx[i] + gs[i];
    }
    if (!gs[i]) return;
    const uint32_t r = rx[i] + brk[i] - 1u;
    const uint32_t nruns = rx[n - 1] + brk[n - 1];
    const int run_end = r + 1u < nruns ? (int)runs[r + 1] : n;
    const int c = cloud[i];
    groups[gx[i]] = make_int4(i, min(i + kWave, run_end), roots[c], roots[c + 1]);
}

static hipError_t knn_groups(wnnc_ctx_s *ctx) {
    const int n = (int)ctx->n;
    hipStream_t st = ctx->stream;
    hipError_t e = ctx->knn_tmp.ensure(5 * (int64_t)n + 1);
    if (e != hipSuccess) return e;
    uint32_t *brk = ctx->knn_tmp.p, *rx = brk + n, *runs = rx + n, *gs = runs + n, *gx = gs + n;
    uint32_t *cnt = gx + n;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_knn_brk, dim3(nb), dim3(256), 0, st, ctx->keys_a.p, n, brk);
    if ((e = exclusive_scan_u32(brk, rx, n, ctx->scan_tmp.p, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_knn_runs, dim3(nb), dim3(256), 0, st, brk, rx, n, runs);
    hipLaunchKernelGGL(k_knn_gflag, dim3(nb), dim3(256), 0, st, brk, rx, runs, n, gs);
    if ((e = exclusive_scan_u32(gs, gx, n, ctx->scan_tmp.p, st)) != hipSuccess) return e;
    // at most one group per point
    if ((e = ctx->knn_groups.ensure(n)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_knn_groups, dim3(nb), dim3(256), 0, st, brk, rx, runs, gs, gx, n,
                       ctx->cloud_of.p, ctx->d_roots.p, ctx->knn_groups.p, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    uint32_t ng = 0;
    if ((e = hipMemcpyAsync(&ng, cnt, sizeof(ng), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    ctx->knn_ngroups = (int)ng;
    return hipSuccess;
}

hipError_t launch_knn(wnnc_ctx_s *ctx) {
    const int n = (int)ctx->n;
    hipError_t e = ctx->knn_idx.ensure((int64_t)n * kK);
    if (e != hipSuccess) return e;
    e = ctx->knn_d2.ensure((int64_t)n * kK);
    if (e != hipSuccess) return e;
    if (ctx->knn_ngroups == 0 && (e = knn_groups(ctx)) != hipSuccess) return e;
    if (ctx->knn_ngroups > 0)
        hipLaunchKernelGGL(k_knn, dim3((unsigned)ctx->knn_ngroups), dim3(kWave), 0, ctx->stream,
                           ctx->pts.p, ctx->cells.p, ctx->topo.p, ctx->knn_groups.p,
                           ctx->d_offsets.p, ctx->cloud_of.p, ctx->knn_ngroups, ctx->knn_idx.p,
                           ctx->knn_d2.p);
    return hipGetLastError();
}

hipError_t launch_knn_features(wnnc_ctx_s *ctx, float *feat, int32_t *nbr_caller) {
    const int n = (int)ctx->n;
    hipError_t e = launch_knn(ctx);
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_features, dim3(nb), dim3(256), 0, ctx->stream, ctx->pts.p, ctx->perm.p,
                       ctx->knn_idx.p, n, feat, nbr_caller);
    return hipGetLastError();
}

}  // namespace wnnc
