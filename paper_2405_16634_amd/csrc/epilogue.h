// Epilogues of the operator walks (Alg. 2 and Alg. 3's per-target updates
// and the per-group reductions behind the step length), shared by the
// traversal, its combining pass and the moment pass that combines split
// walks itself.
#pragma once

#include <float.h>

#include "common.h"
#include "wave.h"

namespace wnnc {

constexpr double kInv4Pi = 0.0795774715459476678844;  // 1 / (4 pi)

// Per-target epilogue from the FP64 sums of target t (sorted position);
// accumulates the target's share of the per-group reductions.  nu receives
// the value written for TR_RHO (rho, 0, 0), TR_R and TR_RESCALE (the
// attribute of the moment pass that follows).
template <int OP, int MODE>
__device__ inline void finish_target(const TravArgs &a, int t, double s, double gx, double gy,
                                     double gz, double &e, double &e2, unsigned &nflip,
                                     float4 &nu) {
    if (MODE == TR_ACCUM) {
        const int64_t j = a.tperm[t];
        a.out[3 * j] = (float)(gx * kInv4Pi + (double)a.gradf[3 * j]);
        a.out[3 * j + 1] = (float)(gy * kInv4Pi + (double)a.gradf[3 * j + 1]);
        a.out[3 * j + 2] = (float)(gz * kInv4Pi + (double)a.gradf[3 * j + 2]);
    } else if (MODE == TR_POSGRAD) {
        // dL/dx = p + g grad F at the target's caller row
        const int64_t j = a.tperm[t];
        const double gj = (double)a.gc[j];
        a.out[3 * j] = (float)(gx * kInv4Pi + gj * (double)a.gradf[3 * j]);
        a.out[3 * j + 1] = (float)(gy * kInv4Pi + gj * (double)a.gradf[3 * j + 1]);
        a.out[3 * j + 2] = (float)(gz * kInv4Pi + gj * (double)a.gradf[3 * j + 2]);
    } else if (MODE == TR_OUT_CALLER) {
        const int64_t j = a.tperm[t];
        if (OP == OP_A) {
            a.out[j] = (float)(s * (kInv4Pi * a.oscale));
        } else {
            const double sg = (OP == OP_G ? -kInv4Pi : kInv4Pi) * a.oscale;  // grad F = -G
            a.out[3 * j] = (float)(gx * sg);
            a.out[3 * j + 1] = (float)(gy * sg);
            a.out[3 * j + 2] = (float)(gz * sg);
        }
    } else if (MODE == TR_RHO) {
        const float rho = (float)(0.5 - s * kInv4Pi);
        a.rho[t] = rho;
        nu = make_float4(rho, 0.f, 0.f, 0.f);
        e += (double)rho * (double)rho;
    } else if (MODE == TR_R) {
        const float rx = (float)(gx * kInv4Pi), ry = (float)(gy * kInv4Pi),
                    rz = (float)(gz * kInv4Pi);
        nu = make_float4(rx, ry, rz, 0.f);
        a.out4[t] = nu;
        e += (double)rx * rx + (double)ry * ry + (double)rz * rz;
    } else if (MODE == TR_TSUM) {
        const double tv = (double)(float)(s * kInv4Pi);
        e += tv * tv;
    } else if (MODE == TR_SCALE) {
        const double tv = (double)(float)(s * kInv4Pi);
        e += tv;
        e2 += tv * tv;
    } else if (MODE == TR_RESCALE) {
        const float4 mu = a.src4[t];
        const double g2 = gx * gx + gy * gy + gz * gz;
        float4 o = mu;
        if (g2 > 0.0 && g2 <= DBL_MAX) {
            // the length kept: |mu| (Alg. 3), or a given area (Sec. 6.1.1)
            const double mn = a.areas ? (double)a.areas[t]
                                      : sqrt((double)mu.x * mu.x + (double)mu.y * mu.y +
                                             (double)mu.z * mu.z);
            const double f = mn / sqrt(g2);
            o = make_float4((float)(gx * f), (float)(gy * f), (float)(gz * f), 0.f);
        }
        a.out4[t] = o;
        nu = o;
        if ((double)mu.x * gx + (double)mu.y * gy + (double)mu.z * gz < 0.0) ++nflip;
    }
}

// Per-group reductions of a wavefront (one group slot), in a fixed order.
template <int MODE>
__device__ inline void finish_group(const TravArgs &a, int sl, int first, int lane, double e,
                                    double e2, unsigned nflip) {
    if (MODE == TR_RESCALE && a.flips) {
        unsigned tot = nflip;
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) tot += __shfl_xor(tot, d, kWave);
        if (lane == 0 && tot) atomicAdd(a.flips + a.tcloud[first], (unsigned long long)tot);
    }
    // (fixed-order scans: reproducible; the last lane holds the sum)
    if (MODE == TR_SCALE) {
        e = wave_scan(e);
        e2 = wave_scan(e2);
        if (lane == kWave - 1) {
            a.partial[sl] = e;
            a.partial[a.nslots + sl] = e2;
        }
    }
    if (MODE == TR_RHO || MODE == TR_R || MODE == TR_TSUM) {
        e = wave_scan(e);
        if (lane == kWave - 1) a.partial[sl] = e;
    }
}

// The sums of one 64-target group walked in parts [pf, pe): the parts' FP32
// sums (component-major, 3 x 64 floats per part) added in part order in
// FP64, kCombineBatch parts' loads in flight before their additions (a part
// is within 2^-24 of the sum of its terms' magnitudes).
constexpr int kCombineBatch = 4;

template <int OP>
__device__ inline void sum_parts(const float *parts, int pf, int pe, int lane, double &s,
                                 double &gx, double &gy, double &gz) {
    for (int p0 = pf; p0 < pe; p0 += kCombineBatch) {
        float v0[kCombineBatch], v1[kCombineBatch], v2[kCombineBatch];
#pragma unroll
        for (int u = 0; u < kCombineBatch; ++u) {
            // (a part past the group's last reads the last one; not added)
            const float *qp = parts + (int64_t)min(p0 + u, pe - 1) * (3 * kWave);
            v0[u] = qp[lane];
            if (OP != OP_A) {
                v1[u] = qp[kWave + lane];
                v2[u] = qp[2 * kWave + lane];
            }
        }
#pragma unroll
        for (int u = 0; u < kCombineBatch; ++u) {
            if (p0 + u < pe) {
                if (OP == OP_A) {
                    s += (double)v0[u];
                } else {
                    gx += (double)v0[u];
                    gy += (double)v1[u];
                    gz += (double)v2[u];
                }
            }
        }
    }
}

}  // namespace wnnc
