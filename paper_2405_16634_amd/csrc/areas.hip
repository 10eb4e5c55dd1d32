// kNN local-area estimate (Sec. 6.1: the areas the paper compares the solved
// |mu_i| with in Table 5, and the fixed areas of the rescale variant).
//
// Per point, from its k nearest neighbours of the same cloud:
//   1. offsets q_j to the neighbours, in FP64 from the FP32 coordinates;
//   2. the tangent plane's normal n: the eigenvector of the smallest
//      eigenvalue of the covariance of the point and its neighbours (cyclic
//      Jacobi rotations on the 3x3 matrix, FP64);
//   3. the in-plane basis e1 = the nearest neighbour's offset projected onto
//      the plane (the next one when that projection is 0), e2 = n x e1;
//   4. the 2-D offsets u_j = (q_j . e1, q_j . e2);
//   5. the area of the origin's Voronoi cell among the u_j (half-planes
//      z . u_j <= |u_j|^2 / 2), clipped to the square [-R, R]^2 with
//      R = max |u_j| so that cells at the edge of an open surface stay
//      bounded.
// Fewer than 2 neighbours (clouds of 1 or 2 points), or no offset with a
// non-zero projection, give area 0.
//
// One thread per point.  The polygon of step 5 is clipped one half-plane at
// a time (Sutherland-Hodgman); its vertices live in LDS, two ping-pong
// buffers per thread laid out [vertex][lane] so that the lanes of a
// wavefront touch consecutive words.
#include <float.h>
#include <math.h>

#include "common.h"
#include "internal.h"

namespace wnnc {

namespace {

constexpr int kAK = 16;                // neighbours computed per point
constexpr int kPolyMax = 4 + kAK + 4;  // vertex capacity: a convex clip adds at most one
constexpr int kAreaBlock = 64;

// One Jacobi rotation zeroing A[p][q] of the symmetric 3x3 A (row-major),
// accumulated into the eigenvector columns of V.
template <int P, int Q>
__device__ inline void jacobi_rotate(double (&A)[9], double (&V)[9]) {
    const double apq = A[P * 3 + Q];
    if (apq == 0.0) return;
    const double theta = (A[Q * 3 + Q] - A[P * 3 + P]) / (2.0 * apq);
    const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
    const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
    double B[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) B[i] = A[i];
    // A' = J^T A J with J the rotation in the (P, Q) plane
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double akp = A[k * 3 + P], akq = A[k * 3 + Q];
        B[k * 3 + P] = c * akp - s * akq;
        B[k * 3 + Q] = s * akp + c * akq;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double bpk = B[P * 3 + k], bqk = B[Q * 3 + k];
        A[P * 3 + k] = c * bpk - s * bqk;
        A[Q * 3 + k] = s * bpk + c * bqk;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (k != P && k != Q) A[k * 3 + P] = A[P * 3 + k], A[k * 3 + Q] = A[Q * 3 + k];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double vkp = V[k * 3 + P], vkq = V[k * 3 + Q];
        V[k * 3 + P] = c * vkp - s * vkq;
        V[k * 3 + Q] = s * vkp + c * vkq;
    }
}

// Unit eigenvector of the smallest eigenvalue of the symmetric 3x3 A.
__device__ inline void smallest_eigvec(double (&A)[9], double &nx, double &ny, double &nz) {
    double V[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int sweep = 0; sweep < 16; ++sweep) {
        const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        const double dia = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (!(off > 1e-32 * dia)) break;
        jacobi_rotate<0, 1>(A, V);
        jacobi_rotate<0, 2>(A, V);
        jacobi_rotate<1, 2>(A, V);
    }
    int m = 0;
    if (A[4] < A[m * 4]) m = 1;
    if (A[8] < A[m * 4]) m = 2;
    nx = V[0 * 3 + m], ny = V[1 * 3 + m], nz = V[2 * 3 + m];
    const double l = sqrt(nx * nx + ny * ny + nz * nz);
    nx /= l, ny /= l, nz /= l;
}

__global__ __launch_bounds__(kAreaBlock) void k_knn_areas(const float4 *__restrict__ pts,
                                                          const uint32_t *__restrict__ perm,
                                                          const int32_t *__restrict__ nbr, int n,
                                                          int k, float *__restrict__ areas) {
    __shared__ double sx[2][kPolyMax][kAreaBlock];
    __shared__ double sy[2][kPolyMax][kAreaBlock];
    const int lane = threadIdx.x;
    const int t = blockIdx.x * kAreaBlock + lane;
    if (t >= n) return;
    const float4 p = pts[t];
    // step 1: offsets (missing neighbours are -1, after the valid ones)
    double qx[kAK], qy[kAK], qz[kAK];
    int m = 0;
#pragma unroll
    for (int i = 0; i < kAK; ++i) {
        const int j = i < k ? nbr[(int64_t)t * kAK + i] : -1;
        qx[i] = qy[i] = qz[i] = 0.0;
        if (j >= 0) {
            const float4 q = pts[j];
            qx[i] = (double)q.x - (double)p.x;
            qy[i] = (double)q.y - (double)p.y;
            qz[i] = (double)q.z - (double)p.z;
            ++m;
        }
    }
    float area = 0.0f;
    if (m >= 2) {
        // step 2: covariance of {0} and the offsets about their mean
        double mx = 0.0, my = 0.0, mz = 0.0;
#pragma unroll
        for (int i = 0; i < kAK; ++i) mx += qx[i], my += qy[i], mz += qz[i];
        const double inv = 1.0 / (m + 1);
        mx *= inv, my *= inv, mz *= inv;
        // the point itself, at offset 0
        double A[9] = {mx * mx, mx * my, mx * mz, 0, my * my, my * mz, 0, 0, mz * mz};
#pragma unroll
        for (int i = 0; i < kAK; ++i) {
            if (i < m) {
                const double dx = qx[i] - mx, dy = qy[i] - my, dz = qz[i] - mz;
                A[0] += dx * dx, A[1] += dx * dy, A[2] += dx * dz;
                A[4] += dy * dy, A[5] += dy * dz, A[8] += dz * dz;
            }
        }
        A[3] = A[1], A[6] = A[2], A[7] = A[5];
        double nx, ny, nz;
        smallest_eigvec(A, nx, ny, nz);
        // step 3: e1 from the first offset with a non-zero projection
        double ex = 0.0, ey = 0.0, ez = 0.0;
        bool have = false;
#pragma unroll
        for (int i = 0; i < kAK; ++i) {
            const double d = qx[i] * nx + qy[i] * ny + qz[i] * nz;
            const double tx = qx[i] - d * nx, ty = qy[i] - d * ny, tz = qz[i] - d * nz;
            const double tl = sqrt(tx * tx + ty * ty + tz * tz);
            if (!have && i < m && tl > 0.0) ex = tx / tl, ey = ty / tl, ez = tz / tl, have = true;
        }
        if (have) {
            const double fx = ny * ez - nz * ey, fy = nz * ex - nx * ez, fz = nx * ey - ny * ex;
            // step 4: 2-D offsets, and the clip square's half-side R
            double R = 0.0;
#pragma unroll
            for (int i = 0; i < kAK; ++i) {
                const double u = qx[i] * ex + qy[i] * ey + qz[i] * ez;
                const double v = qx[i] * fx + qy[i] * fy + qz[i] * fz;
                qx[i] = u, qy[i] = v;
                if (i < m) R = fmax(R, sqrt(u * u + v * v));
            }
            // step 5: the square, counter-clockwise, then one clip per offset
            int cur = 0, cnt = 4;
            sx[0][0][lane] = -R, sy[0][0][lane] = -R;
            sx[0][1][lane] = R, sy[0][1][lane] = -R;
            sx[0][2][lane] = R, sy[0][2][lane] = R;
            sx[0][3][lane] = -R, sy[0][3][lane] = R;
#pragma unroll
            for (int i = 0; i < kAK; ++i) {
                const double ux = qx[i], uy = qy[i];
                const double h = 0.5 * (ux * ux + uy * uy);
                if (i >= m || !(h > 0.0) || cnt < 3) continue;
                const int nxt = cur ^ 1;
                int out = 0;
                double px = sx[cur][cnt - 1][lane], py = sy[cur][cnt - 1][lane];
                double fp = px * ux + py * uy - h;
                for (int v = 0; v < cnt; ++v) {
                    const double cx = sx[cur][v][lane], cy = sy[cur][v][lane];
                    const double fc = cx * ux + cy * uy - h;
                    // edge (p -> c): the crossing first, then c if inside
                    if ((fp < 0.0 && fc > 0.0) || (fp > 0.0 && fc < 0.0)) {
                        const double s = fp / (fp - fc);
                        if (out < kPolyMax) {
                            sx[nxt][out][lane] = px + s * (cx - px);
                            sy[nxt][out][lane] = py + s * (cy - py);
                            ++out;
                        }
                    }
                    if (fc <= 0.0 && out < kPolyMax) {
                        sx[nxt][out][lane] = cx, sy[nxt][out][lane] = cy;
                        ++out;
                    }
                    px = cx, py = cy, fp = fc;
                }
                cur = nxt, cnt = out;
            }
            // shoelace
            double a2 = 0.0;
            if (cnt >= 3) {
                double px = sx[cur][cnt - 1][lane], py = sy[cur][cnt - 1][lane];
                for (int v = 0; v < cnt; ++v) {
                    const double cx = sx[cur][v][lane], cy = sy[cur][v][lane];
                    a2 += px * cy - cx * py;
                    px = cx, py = cy;
                }
            }
            area = (float)(0.5 * fabs(a2));
        }
    }
    areas[perm[t]] = area;
}

}  // namespace

hipError_t launch_knn_areas(wnnc_ctx_s *ctx, int k, float *areas_out) {
    const int n = (int)ctx->n;
    hipLaunchKernelGGL(k_knn_areas, dim3((unsigned)((n + kAreaBlock - 1) / kAreaBlock)),
                       dim3(kAreaBlock), 0, ctx->stream, ctx->pts.p, ctx->perm.p,
                       ctx->knn_idx.p, n, k, areas_out);
    return hipGetLastError();
}

}  // namespace wnnc
