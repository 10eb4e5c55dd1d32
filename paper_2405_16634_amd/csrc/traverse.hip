// Treecode traversal (Sec. 3.5, Alg. 4) for the three operators.
//
// One lane per target; a wavefront holds 64 Morton-consecutive targets and
// walks the pre-order node array once.  Every lane keeps its own Alg. 4
// decisions: at node B, a lane that is still "inside" (has not replaced an
// ancestor of B by its representative) tests |x - x_B| > c * width(B) and,
// if so, adds the representative term; lanes that fail the test need B's
// children (or, at a leaf, B's points).  The wavefront descends into B when
// any lane needs it, with the set of such lanes pushed on a per-depth mask
// stack (held one mask per lane in two VGPRs, read with readlane), and skips
// the subtree otherwise.  A single-point leaf's representative is its point,
// so such a leaf is evaluated as a representative by every inside lane.
//
// Node records are read with scalar loads: the node index is uniform across
// the wavefront.  The 1/(4 pi) factor is applied in the epilogue.
#include <float.h>

#include "common.h"
#include "internal.h"

namespace wnnc {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Loads through the constant address space: uniform addresses become SMEM
// loads (the arrays are not written during the kernel).
__device__ inline int4 ldc_i4(const int4 *p) {
    v4i v = *(const __attribute__((address_space(4))) v4i *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ inline float4 ldc_f4(const float4 *p) {
    v4f v = *(const __attribute__((address_space(4))) v4f *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ inline float ldc_f(const float *p) {
    return *(const __attribute__((address_space(4))) float *)p;
}

constexpr float kInv4Pi = 0.0795774715459476678844f;

// Pair term without the 1/(4 pi) factor.  d = target - source, r2 = |d|^2.
//   A  : -(d . nu) / r^3
//   A^T: nu d / r^3                      (nu scalar, in v.x)
//   G  : nu / r^3 - 3 (d . nu) d / r^5
// Kept only when r >= w and r > 0 (Sec. 3.4).
template <int OP>
__device__ inline void pair_term(float dx, float dy, float dz, float r2, float4 v, float w2,
                                 float &s, float &gx, float &gy, float &gz) {
    const bool keep = (r2 >= w2) && (r2 > 0.0f);
    // hardware reciprocal square root (about 1 ulp); r2 below the smallest
    // normal only occurs for pairs that the cutoff removes when w > 0
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float ri2 = ri * ri;
    const float ri3 = ri2 * ri;
    if (OP == OP_A) {
        const float dm = fmaf(dx, v.x, fmaf(dy, v.y, dz * v.z));
        const float t = -dm * ri3;
        s += keep ? t : 0.0f;
    } else if (OP == OP_AT) {
        const float f = v.x * ri3;
        gx += keep ? f * dx : 0.0f;
        gy += keep ? f * dy : 0.0f;
        gz += keep ? f * dz : 0.0f;
    } else {
        const float dm = fmaf(dx, v.x, fmaf(dy, v.y, dz * v.z));
        const float c5 = 3.0f * dm * (ri3 * ri2);
        gx += keep ? fmaf(v.x, ri3, -c5 * dx) : 0.0f;
        gy += keep ? fmaf(v.y, ri3, -c5 * dy) : 0.0f;
        gz += keep ? fmaf(v.z, ri3, -c5 * dz) : 0.0f;
    }
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Block sum of one double per thread in a fixed order; valid in thread 0.
__device__ inline double block_sum(double v) {
    __shared__ double ws[kTravBlock / kWave];
    __syncthreads();  // a previous call may still be reading ws
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    if (lane == 0) ws[wv] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kTravBlock / kWave; ++k) t += ws[k];
    return t;
}

template <int OP, int MODE, bool COUNT>
__global__ __launch_bounds__(kTravBlock) void k_traverse(TravArgs a) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous range of Morton-ordered targets so its L2 sees one region.
    const int G = gridDim.x, b = blockIdx.x;
    const int q = G >> 3, r = G & 7, x = b & 7;
    const int lb = x * q + (x < r ? x : r) + (b >> 3);
    const int t = (lb * (kTravBlock / kWave) + wv) * kWave + lane;
    const bool valid = t < a.n;

    float tx = 0.f, ty = 0.f, tz = 0.f;
    if (valid) {
        const float4 p = a.pts[t];
        tx = p.x, ty = p.y, tz = p.z;
    }
    float s = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
    uint32_t cnt = 0;
    const unsigned long long act0 = __ballot(valid);
    if (act0 != 0ull) {
        // mask stack: lane d holds the mask of lanes inside at depth d
        uint32_t mlo = lane == 0 ? (uint32_t)act0 : 0u;
        uint32_t mhi = lane == 0 ? (uint32_t)(act0 >> 32) : 0u;
        int node = 0;
        const int m = a.m;
        while (node < m) {
            const float4 P = ldc_f4(a.mom + 2 * node);
            const float4 V = ldc_f4(a.mom + 2 * node + 1);
            const int flags = __float_as_int(P.w);
            const int skip = __float_as_int(V.w);
            if (flags & kRecZero) {  // every attribute in the node is zero
                node = skip;
                continue;
            }
            const int depth = flags & 15;
            const unsigned long long act =
                (unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)mlo, depth) |
                ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)mhi, depth) << 32);
            const bool me = (act >> lane) & 1ull;
            const float dx = tx - P.x, dy = ty - P.y, dz = tz - P.z;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const bool far = me && ((flags & kRecSingle) || r2 > a.thr2[depth]);
            if (far) {
                pair_term<OP>(dx, dy, dz, r2, V, a.w2, s, gx, gy, gz);
                if (COUNT) ++cnt;
            }
            const unsigned long long open = __ballot(me && !far);
            if (open == 0ull) {
                node = skip;
                continue;
            }
            if (flags & kRecLeaf) {
                // several points in a depth-D cell: direct sum for the lanes
                // that did not accept the representative
                const int4 tp = ldc_i4(a.topo + node);
                const bool mine = (open >> lane) & 1ull;
                for (int j = tp.y; j < tp.z; ++j) {
                    const float4 Q = ldc_f4(a.pts + j);
                    float4 S;
                    if (OP == OP_AT)
                        S = make_float4(ldc_f(a.srcs + j), 0.f, 0.f, 0.f);
                    else
                        S = ldc_f4(a.src4 + j);
                    if (mine) {
                        const float ex = tx - Q.x, ey = ty - Q.y, ez = tz - Q.z;
                        const float e2 = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
                        pair_term<OP>(ex, ey, ez, e2, S, a.w2, s, gx, gy, gz);
                        if (COUNT) ++cnt;
                    }
                }
                node = skip;
            } else {
                if (lane == depth + 1) {
                    mlo = (uint32_t)open;
                    mhi = (uint32_t)(open >> 32);
                }
                node = node + 1;
            }
        }
    }

    // epilogues
    if (MODE == TR_OUT_CALLER) {
        if (valid) {
            const int64_t j = a.perm[t];
            if (OP == OP_A) {
                a.out[j] = s * kInv4Pi;
            } else {
                const float sg = OP == OP_G ? -kInv4Pi : kInv4Pi;  // grad F = -G
                a.out[3 * j] = gx * sg;
                a.out[3 * j + 1] = gy * sg;
                a.out[3 * j + 2] = gz * sg;
            }
        }
    } else if (MODE == TR_RHO) {
        double e = 0.0;
        if (valid) {
            const float rho = 0.5f - s * kInv4Pi;
            a.rho[t] = rho;
            e = (double)rho * (double)rho;
        }
        e = block_sum(e);
        if (threadIdx.x == 0) a.partial[lb] = e;
    } else if (MODE == TR_R) {
        double e = 0.0;
        if (valid) {
            const float rx = gx * kInv4Pi, ry = gy * kInv4Pi, rz = gz * kInv4Pi;
            a.out4[t] = make_float4(rx, ry, rz, 0.f);
            e = (double)rx * rx + (double)ry * ry + (double)rz * rz;
        }
        e = block_sum(e);
        if (threadIdx.x == 0) a.partial[lb] = e;
    } else if (MODE == TR_TSUM) {
        double e = 0.0;
        if (valid) {
            const double tv = (double)(s * kInv4Pi);
            e = tv * tv;
        }
        e = block_sum(e);
        if (threadIdx.x == 0) a.partial[lb] = e;
    } else if (MODE == TR_RESCALE) {
        if (valid) {
            const float4 mu = a.src4[t];
            const double g2 = (double)gx * gx + (double)gy * gy + (double)gz * gz;
            float4 o = mu;
            if (g2 > 0.0 && g2 <= DBL_MAX) {
                const double mn = sqrt((double)mu.x * mu.x + (double)mu.y * mu.y + (double)mu.z * mu.z);
                const double f = mn / sqrt(g2);
                o = make_float4((float)(gx * f), (float)(gy * f), (float)(gz * f), 0.f);
            }
            a.out4[t] = o;
        }
    }
    if (COUNT) {
        double c = block_sum((double)cnt);
        if (threadIdx.x == 0) atomicAdd(a.pairs + OP, (unsigned long long)c);
    }
}

int trav_blocks(int64_t n) { return (int)((n + kTravBlock - 1) / kTravBlock); }

template <int OP, int MODE>
static void launch_one(bool count, const TravArgs &a, hipStream_t st) {
    const dim3 grid((unsigned)trav_blocks(a.n)), block(kTravBlock);
    if (count)
        hipLaunchKernelGGL((k_traverse<OP, MODE, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((k_traverse<OP, MODE, false>), grid, block, 0, st, a);
}

hipError_t launch_traverse(wnnc_ctx_s *ctx, Op op, TravMode mode, bool count, const TravArgs &a) {
    hipStream_t st = ctx->stream;
    if (op == OP_A) {
        if (mode == TR_OUT_CALLER)
            launch_one<OP_A, TR_OUT_CALLER>(count, a, st);
        else if (mode == TR_RHO)
            launch_one<OP_A, TR_RHO>(count, a, st);
        else if (mode == TR_TSUM)
            launch_one<OP_A, TR_TSUM>(count, a, st);
        else
            return hipErrorInvalidValue;
    } else if (op == OP_AT) {
        if (mode == TR_OUT_CALLER)
            launch_one<OP_AT, TR_OUT_CALLER>(count, a, st);
        else if (mode == TR_R)
            launch_one<OP_AT, TR_R>(count, a, st);
        else
            return hipErrorInvalidValue;
    } else {
        if (mode == TR_OUT_CALLER)
            launch_one<OP_G, TR_OUT_CALLER>(count, a, st);
        else if (mode == TR_RESCALE)
            launch_one<OP_G, TR_RESCALE>(count, a, st);
        else
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace wnnc
