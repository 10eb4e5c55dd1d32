// The per-call moment pass: nu-representatives of every octree node
// (Sec. 4.5, eqs. for the node representative location and vector):
//   W_B = sum_{i in B} |nu_i|,  x_B = sum |nu_i| x_i / W_B,  nu_B = sum nu_i.
//
// Nodes are contiguous ranges of the Morton-sorted points.  The points are
// cut into chunks of kChunk; one workgroup per chunk forms FP64 inclusive
// prefix sums of (|nu|, |nu| x, nu) and finishes every node that lies inside
// its chunk as a difference of two prefixes.  Nodes that cross a chunk
// boundary ("straddlers") receive a head partial from their first chunk, a
// tail partial from their last, and the totals of the chunks in between in a
// second launch (one wavefront per straddler, the whole workgroup for one
// that spans more than a wavefront's worth of chunks).  All sums run in a
// fixed order, so the moments are bitwise reproducible from run to run.
// When the attribute is the output of a walk split into parts, the chunk
// pass can also run that walk's combining pass first (k_moments_comb).
//
// With a far field of order 1 or 2 (an extension: the Taylor expansion of
// the pair term about x_B) the same pass also sums raw moments about the
// origin in FP64 and writes the central ones about x_B (d = x - x_B) by the
// parallel-axis shift.  For a vector attribute only the parts symmetric in
// all indices are needed (the Taylor terms contract them with derivatives
// of 1/r), and those shift among themselves:
//   M1_kn = sym sum x_k nu_n,  M2_knl = sym sum x_k x_n nu_l,
//   D_kn  = M1_kn - sym(x_Bk nu_Bn),
//   Q_knl = M2_knl - (2/3)(x_Bk M1_nl + x_Bn M1_kl + x_Bl M1_kn)
//           + sym(x_Bk x_Bn nu_Bl),
// with sym(a_k b_n) = (a_k b_n + a_n b_k)/2 and sym(a_k a_n b_l) =
// (a_k a_n b_l + a_k a_l b_n + a_n a_l b_k)/3.  For a scalar rho:
//   p_k = sum rho x_k - x_Bk rho_B,
//   q_kn = sum rho x_k x_n - x_Bk P_n - x_Bn P_k + x_Bk x_Bn rho_B (P = sum rho x).
// (In FP64 the shift loses about (1/width)^2 of relative precision: 1e-8 at
// the deepest level, far below the FP32 the moments are stored in.)
#include <float.h>

#include "common.h"
#include "epilogue.h"
#include "internal.h"
#include "wave.h"

namespace wnnc {

// values per point: |nu|, |nu| x (3), nu (3); with HI also, for a vector
// attribute, M1 (6 pairs) and M2 (10 triples), for a scalar one rho x_k (3)
// and rho x_k x_n (6 pairs)
template <bool HI>
constexpr int mom_vals() { return HI ? kMomHi : kMomBase; }
constexpr int kPairK[6] = {0, 0, 0, 1, 1, 2};
constexpr int kPairN[6] = {0, 1, 2, 1, 2, 2};
constexpr int kTriK[10] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 2};
constexpr int kTriN[10] = {0, 0, 0, 1, 1, 2, 1, 1, 2, 2};
constexpr int kTriL[10] = {0, 1, 2, 1, 2, 2, 1, 2, 2, 2};

// The pair index of (k, n) in either order.
__device__ constexpr int pair_of(int k, int n) {
    return k > n ? pair_of(n, k) : (k == 0 ? n : (k == 1 ? 2 + n : 5));
}

// The raw far-field values of one point (slots kMomBase..kMomHi-1).
__device__ inline void raw_hi(const float4 x, double n0, double n1, double n2, bool scalar,
                              double *v) {
    const double xs[3] = {(double)x.x, (double)x.y, (double)x.z};
    const double ns[3] = {n0, n1, n2};
    if (scalar) {
#pragma unroll
        for (int k = 0; k < 3; ++k) v[kMomBase + k] = xs[k] * n0;
#pragma unroll
        for (int p = 0; p < 6; ++p) v[kMomBase + 3 + p] = xs[kPairK[p]] * xs[kPairN[p]] * n0;
#pragma unroll
        for (int i = kMomBase + 9; i < kMomHi; ++i) v[i] = 0.0;
        return;
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const int k = kPairK[p], n = kPairN[p];
        v[kMomBase + p] = 0.5 * (xs[k] * ns[n] + xs[n] * ns[k]);
    }
#pragma unroll
    for (int t = 0; t < 10; ++t) {
        const int k = kTriK[t], n = kTriN[t], l = kTriL[t];
        v[kMomBase + 6 + t] = (xs[k] * xs[n] * ns[l] + xs[k] * xs[l] * ns[n] +
                               xs[n] * xs[l] * ns[k]) * (1.0 / 3.0);
    }
}

// Stores three floats (one 12-byte store at a 16-byte aligned address).
__device__ inline void st3(float4 *p, float x, float y, float z) {
    float *q = (float *)p;
    q[0] = x;
    q[1] = y;
    q[2] = z;
}

// Node record: x_B = X / W and nu_B in FP32 beside the node's flags and skip
// pointer (written with the tree), so that the traversal needs one 64-byte
// load per node.  A single-point leaf's representative is its point, so
// only its nu_B is written here (12 bytes); its position, flags and
// threshold (-1: every target takes it) are written with the tree.  A node
// whose weight W is zero (every attribute in it is zero) gets threshold -1
// as well: every target takes it, with nu_B = 0 an exact zero term, and
// none descends into it.
template <bool HI>
__device__ inline void write_moment(const MomArgs &a, int node, int depth, bool single,
                                    const double *s) {
    const double W = s[0];
    float4 *rec = a.mom + (int64_t)kRecStride * node;
    st3(rec + 1, (float)s[4], (float)s[5], (float)s[6]);
    if (!single) {
        float hx = 0.f, hy = 0.f, hz = 0.f;
        float4 lo = make_float4(0.f, 0.f, 0.f, a.thr2[depth]);
        if (W > 0.0) {
            const double x = s[1] / W, y = s[2] / W, z = s[3] / W;
            hx = (float)x, hy = (float)y, hz = (float)z;
            lo = make_float4((float)(x - (double)hx), (float)(y - (double)hy),
                             (float)(z - (double)hz), lo.w);
        } else {
            lo.w = -1.0f;
        }
        st3(rec, hx, hy, hz);
        rec[2] = lo;
    }
    if (a.wout) a.wout[node] = W > 0.0 ? fmaxf((float)W, FLT_MIN) : 0.f;
    if (HI) {
        // central moments about x_B (0 for a node that carries nothing)
        const bool live = W > 0.0;
        const double xb[3] = {live ? s[1] / W : 0.0, live ? s[2] / W : 0.0,
                              live ? s[3] / W : 0.0};
        const double nb[3] = {s[4], s[5], s[6]};
        const double *m = s + kMomBase;
        float *h = a.momhi + (int64_t)kHiStride * node;
        if (a.scalar) {
            double q[6], tr = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) h[k] = live ? (float)(m[k] - xb[k] * nb[0]) : 0.f;
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const int k = kPairK[p], n = kPairN[p];
                q[p] = m[3 + p] - xb[k] * m[n] - xb[n] * m[k] + xb[k] * xb[n] * nb[0];
                if (k == n) tr += q[p];
                h[3 + p] = live ? (float)q[p] : 0.f;
            }
            h[9] = live ? (float)tr : 0.f;
        } else {
            double D[6], Q[10];
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const int k = kPairK[p], n = kPairN[p];
                D[p] = m[p] - 0.5 * (xb[k] * nb[n] + xb[n] * nb[k]);
            }
#pragma unroll
            for (int t = 0; t < 10; ++t) {
                const int k = kTriK[t], n = kTriN[t], l = kTriL[t];
                Q[t] = m[6 + t] -
                       (2.0 / 3.0) * (xb[k] * m[pair_of(n, l)] + xb[n] * m[pair_of(k, l)] +
                                      xb[l] * m[pair_of(k, n)]) +
                       (xb[k] * xb[n] * nb[l] + xb[k] * xb[l] * nb[n] + xb[n] * xb[l] * nb[k]) *
                           (1.0 / 3.0);
            }
#pragma unroll
            for (int p = 0; p < 6; ++p) h[p] = live ? (float)D[p] : 0.f;
            h[6] = live ? (float)(D[0] + D[3] + D[5]) : 0.f;
#pragma unroll
            for (int t = 0; t < 10; ++t) h[7 + t] = live ? (float)Q[t] : 0.f;
            // e_m = sum_k Q_(k,k,m): triples (0,0,m) (1,1,m) (2,2,m) sorted
            h[17] = live ? (float)(Q[0] + Q[3] + Q[5]) : 0.f;  // 000 011 022
            h[18] = live ? (float)(Q[1] + Q[6] + Q[8]) : 0.f;  // 001 111 122
            h[19] = live ? (float)(Q[2] + Q[7] + Q[9]) : 0.f;  // 002 112 222
        }
    }
}

// The operator walk whose output a combining moment pass reads.
template <int MODE>
struct CombOf {
    static constexpr int op = MODE == MOM_COMB_RHO ? OP_A : (MODE == MOM_COMB_R ? OP_AT : OP_G);
    static constexpr int mode =
        MODE == MOM_COMB_RHO ? TR_RHO : (MODE == MOM_COMB_R ? TR_R : TR_RESCALE);
};

// One chunk (the workgroup's): for the MOM_COMB_* modes ta is the walk's
// arguments, else null.
template <int MODE, bool HI>
__device__ __forceinline__ void chunk_body(const MomArgs &a, const TravArgs *ta) {
    constexpr bool COMB = MODE >= MOM_COMB_RHO;
    constexpr int kMomVals = mom_vals<HI>();
    __shared__ double P[kMomVals][kChunk];
    __shared__ double wtot[kMomVals][kChunk / kWave];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    const int c = blockIdx.x;
    const int c0 = c * kChunk;
    const int cE = min(c0 + kChunk, a.n);
    const int cnt = cE - c0;
    const int i = c0 + tid;
    // the nodes started inside this chunk, and the first one of this thread:
    // loaded first, so that they arrive while the prefix sums are formed
    const int nlo = (int)a.node_off[c0];
    const int nhi = (int)a.node_off[cE];
    const int tlo = (int)a.tail_off[c], thi = (int)a.tail_off[c + 1];
    // (unconditional loads at indices clamped to the arrays: no wait for
    // them inside a branch): this thread's first node, its second one (on
    // the benchmark cloud a chunk of 512 points starts about 950 nodes, so
    // nearly every node is one of these two) and its first straddler ending
    // in this chunk
    const int n0 = max(min(nlo + tid, nhi - 1), 0);
    const int2 t0 = a.mnode[n0];
    const int n1 = max(min(nlo + tid + kChunk, nhi - 1), 0);
    const int2 t1 = a.mnode[n1];
    const int2 tq0 = a.tail_list[max(min(tlo + tid, thi - 1), 0)];

    // (MOM_COMB_*) the walk's combining pass for this wavefront's 64-point
    // group if the group was walked in parts: its parts' sums in part order,
    // then the walk's epilogue (output, per-group reduction), as k_combine
    // does it
    float4 cnu = make_float4(0.f, 0.f, 0.f, 0.f);
    bool combined = false;
    if constexpr (COMB) {
        const int g = (c0 >> 6) + wv;  // (wavefront-uniform)
        if (g < a.ngroups) {
            const int2 pr = a.gtab[g];
            if (pr.y > pr.x) {
                constexpr int OP = CombOf<MODE>::op, TM = CombOf<MODE>::mode;
                double s = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
                sum_parts<OP>(ta->parts, pr.x, pr.y, lane, s, gx, gy, gz);
                double e = 0.0, e2 = 0.0;
                unsigned nflip = 0;
                if (i < a.n) finish_target<OP, TM>(*ta, i, s, gx, gy, gz, e, e2, nflip, cnu);
                finish_group<TM>(*ta, g, g * kWave, lane, e, e2, nflip);
                combined = true;
            }
        }
    }

    double v[kMomVals];
#pragma unroll
    for (int k = 0; k < kMomVals; ++k) v[k] = 0.0;
    if (i < a.n) {
        const float4 x = a.pts[i];
        float nu0 = 0.f, nu1 = 0.f, nu2 = 0.f;
        bool scalar = false;
        if constexpr (COMB) {
            // (a whole walk wrote its output itself)
            if (!combined) {
                if (MODE == MOM_COMB_RHO) cnu.x = ta->rho[i];
                else cnu = ta->out4[i];
            }
            nu0 = cnu.x, nu1 = cnu.y, nu2 = cnu.z;
            scalar = MODE == MOM_COMB_RHO;
        } else if (MODE == MOM_VEC_SORTED) {
            const float4 q = a.src4[i];
            nu0 = q.x, nu1 = q.y, nu2 = q.z;
        } else if (MODE == MOM_SCALAR_SORTED) {
            nu0 = a.srcs[i];
            scalar = true;
        } else if (MODE == MOM_VEC_CALLER) {
            const int64_t j = a.perm[i];
            const float sg = a.csig ? a.csig[j] : 1.0f;
            nu0 = a.cn[3 * j] * sg, nu1 = a.cn[3 * j + 1] * sg, nu2 = a.cn[3 * j + 2] * sg;
            a.out4[i] = make_float4(nu0, nu1, nu2, 0.f);
        } else if (MODE == MOM_SCALAR_CALLER) {
            nu0 = a.cs[a.perm[i]];
            a.outs[i] = nu0;
            scalar = true;
        } else if (MODE == MOM_AXPY) {
            const float al = (float)a.alpha[a.cloud[i]];
            const float4 q = a.src4[i], r = a.r4[i];
            nu0 = fmaf(al, r.x, q.x), nu1 = fmaf(al, r.y, q.y), nu2 = fmaf(al, r.z, q.z);
            a.out4[i] = make_float4(nu0, nu1, nu2, 0.f);
        } else {  // MOM_CONST_HALF
            nu0 = 0.5f;
            a.outs[i] = nu0;
            scalar = true;
        }
        const double d0 = nu0, d1 = nu1, d2 = nu2;
        const double w = scalar ? fabs(d0) : sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        v[0] = w;
        v[1] = w * (double)x.x;
        v[2] = w * (double)x.y;
        v[3] = w * (double)x.z;
        v[4] = d0;
        v[5] = d1;
        v[6] = d2;
        if (HI) raw_hi(x, d0, d1, d2, scalar, v);
    }
    // inclusive scan over the chunk: within each wavefront, then wave totals
#pragma unroll
    for (int k = 0; k < kMomVals; ++k) v[k] = wave_scan(v[k]);
    if (lane == kWave - 1) {
#pragma unroll
        for (int k = 0; k < kMomVals; ++k) wtot[k][wv] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kMomVals; ++k) {
        double base = 0.0;
        for (int w = 0; w < wv; ++w) base += wtot[k][w];
        P[k][tid] = base + v[k];
    }
    __syncthreads();

    // chunk totals slot-major (slot k of chunk c at k * nchunks + c), so that
    // the straddler pass reads consecutive chunks with one coalesced load
    if (tid < kMomVals) a.chunk_tot[(int64_t)tid * gridDim.x + c] = P[tid][cnt - 1];

    // nodes started inside this chunk: the thread's first two from the
    // loads above, any further ones loaded here (their fields are passed as
    // scalars: a selection between whole vectors would keep them in
    // private memory)
    auto node = [&](int nd, int tb, int te) {
        const int b = tb - c0;
        double s[kMomVals];
        if (te >= 0) {
            const int end = te & kMnodeEndMask;
            const int e = end - c0 - 1;
#pragma unroll
            for (int k = 0; k < kMomVals; ++k) s[k] = P[k][e] - (b > 0 ? P[k][b - 1] : 0.0);
            write_moment<HI>(a, nd, te >> kMnodeEndBits, end - tb == 1, s);
        } else {
            const int sl = -1 - te;
#pragma unroll
            for (int k = 0; k < kMomVals; ++k)
                a.head[kMomSlots * sl + k] = P[k][cnt - 1] - (b > 0 ? P[k][b - 1] : 0.0);
        }
    };
    if (nlo + tid < nhi) node(nlo + tid, t0.x, t0.y);
    if (nlo + tid + kChunk < nhi) node(nlo + tid + kChunk, t1.x, t1.y);
    for (int nd = nlo + tid + 2 * kChunk; nd < nhi; nd += kChunk) {
        const int2 t = a.mnode[nd];
        node(nd, t.x, t.y);
    }
    // straddlers whose range ends inside this chunk
    auto tail = [&](int sl, int te) {
        const int e = te - c0 - 1;
#pragma unroll
        for (int k = 0; k < kMomVals; ++k) a.tail[kMomSlots * sl + k] = P[k][e];
    };
    if (tlo + tid < thi) tail(tq0.x, tq0.y);
    for (int q = tlo + tid + kChunk; q < thi; q += kChunk) {
        const int2 tq = a.tail_list[q];
        tail(tq.x, tq.y);
    }
}

template <int MODE, bool HI>
__global__ __launch_bounds__(kChunk) void k_moments_chunk(MomArgs a) {
    chunk_body<MODE, HI>(a, nullptr);
}

// The chunk pass that also runs the combining pass of the walk launched
// before it (MOM_COMB_*; without the far field).
template <int MODE>
__global__ __launch_bounds__(kChunk) void k_moments_comb(MomArgs a, TravArgs ta) {
    chunk_body<MODE, false>(a, &ta);
}

// Straddlers: head + totals of the chunks in between + tail.  A straddler
// with at most a wavefront's worth of chunks in between is summed by one
// wavefront, one chunk total per lane; a wide one (the nodes near the root,
// numbered first) by a whole workgroup of its own (the first n_wide
// workgroups), so that every straddler's loads are in flight at once.  The loads of a
// straddler's topology, head and tail do not depend on each other.  The
// order of the additions is fixed (a DPP scan within a wavefront,
// wavefronts in order).
constexpr int kStradBlock = 512;
constexpr int kStradWaves = kStradBlock / kWave;

template <bool HI>
__global__ __launch_bounds__(kStradBlock) void k_moments_strad(MomArgs a) {
    constexpr int kMomVals = mom_vals<HI>();
    __shared__ double red[kMomVals][kStradWaves];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    const int nchunks = (a.n + kChunk - 1) / kChunk;
    // (the wide straddlers are slots 0 .. n_wide - 1)
    const bool wide = (int)blockIdx.x < a.n_wide;
    const int sl = wide ? (int)blockIdx.x
                        : a.n_wide + ((int)blockIdx.x - a.n_wide) * kStradWaves + wv;
    if (sl >= a.n_strad) return;  // (never in a wide workgroup)
    const int4 t = a.strad_topo[sl];
    const int nd = a.strad_node[sl];
    double hd[kMomVals], tl[kMomVals];
#pragma unroll
    for (int k = 0; k < kMomVals; ++k) hd[k] = tl[k] = 0.0;
    // the thread that writes the record: the last lane of a wavefront (where
    // its scan ends), thread 0 of a wide straddler's workgroup
    const bool writer = wide ? tid == 0 : lane == kWave - 1;
    if (writer) {
#pragma unroll
        for (int k = 0; k < kMomVals; ++k) {
            hd[k] = a.head[kMomSlots * sl + k];
            tl[k] = a.tail[kMomSlots * sl + k];
        }
    }
    const int cb = t.y / kChunk, ce = (t.z - 1) / kChunk;
    double s[kMomVals];
#pragma unroll
    for (int k = 0; k < kMomVals; ++k) s[k] = 0.0;
    for (int c = cb + 1 + (wide ? tid : lane); c < ce; c += wide ? kStradBlock : kWave) {
#pragma unroll
        for (int k = 0; k < kMomVals; ++k) s[k] += a.chunk_tot[(int64_t)k * nchunks + c];
    }
    // the wavefront's sum in its last lane (a fixed-order DPP scan)
#pragma unroll
    for (int k = 0; k < kMomVals; ++k) s[k] = wave_scan(s[k]);
    if (wide) {
        if (lane == kWave - 1) {
#pragma unroll
            for (int k = 0; k < kMomVals; ++k) red[k][wv] = s[k];
        }
        __syncthreads();
        if (tid == 0) {
#pragma unroll
            for (int k = 0; k < kMomVals; ++k) {
                double m = 0.0;
                for (int v = 0; v < kStradWaves; ++v) m += red[k][v];
                s[k] = m;
            }
        }
    }
    if (writer) {
        double tot[kMomVals];
#pragma unroll
        for (int k = 0; k < kMomVals; ++k) tot[k] = (hd[k] + s[k]) + tl[k];
        write_moment<HI>(a, nd, topo_depth(t.w), false, tot);
    }
}

// The straddler pass (the call's last launch).
template <bool HI>
hipError_t launch_strad(wnnc_ctx_s *ctx, const MomArgs &a) {
    const unsigned nb =
        (unsigned)(a.n_wide + (a.n_strad - a.n_wide + kStradWaves - 1) / kStradWaves);
    return launch_k(ctx->lev, true, k_moments_strad<HI>, dim3(nb), dim3(kStradBlock),
                    ctx->stream, a);
}

template <bool HI>
hipError_t launch_moments_t(wnnc_ctx_s *ctx, MomMode mode, const MomArgs &a) {
    const unsigned nchunks = (unsigned)((a.n + kChunk - 1) / kChunk);
    const dim3 grid(nchunks), block(kChunk);
    auto &ev = ctx->lev;
    hipStream_t st = ctx->stream;
    // the straddler pass, when there is one, is the call's last launch
    const bool last = a.n_strad <= 0;
    hipError_t e = hipErrorInvalidValue;
    switch (mode) {
        case MOM_VEC_SORTED:
            e = launch_k(ev, last, k_moments_chunk<MOM_VEC_SORTED, HI>, grid, block, st, a);
            break;
        case MOM_SCALAR_SORTED:
            e = launch_k(ev, last, k_moments_chunk<MOM_SCALAR_SORTED, HI>, grid, block, st, a);
            break;
        case MOM_VEC_CALLER:
            e = launch_k(ev, last, k_moments_chunk<MOM_VEC_CALLER, HI>, grid, block, st, a);
            break;
        case MOM_SCALAR_CALLER:
            e = launch_k(ev, last, k_moments_chunk<MOM_SCALAR_CALLER, HI>, grid, block, st, a);
            break;
        case MOM_AXPY:
            e = launch_k(ev, last, k_moments_chunk<MOM_AXPY, HI>, grid, block, st, a);
            break;
        case MOM_CONST_HALF:
            e = launch_k(ev, last, k_moments_chunk<MOM_CONST_HALF, HI>, grid, block, st, a);
            break;
        default:
            break;
    }
    if (e != hipSuccess || last) return e;
    return launch_strad<HI>(ctx, a);
}

hipError_t launch_moments_comb(wnnc_ctx_s *ctx, MomMode mode, const MomArgs &args,
                               const TravArgs &ta) {
    MomArgs a = args;
    a.scalar = mode == MOM_COMB_RHO;
    if (a.order > 0 || !a.gtab || ta.tpl != 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.n + kChunk - 1) / kChunk)), block(kChunk);
    const bool last = a.n_strad <= 0;
    hipError_t e = hipErrorInvalidValue;
    switch (mode) {
        case MOM_COMB_RHO:
            e = launch_k(ctx->lev, last, k_moments_comb<MOM_COMB_RHO>, grid, block, ctx->stream, a,
                         ta);
            break;
        case MOM_COMB_R:
            e = launch_k(ctx->lev, last, k_moments_comb<MOM_COMB_R>, grid, block, ctx->stream, a,
                         ta);
            break;
        case MOM_COMB_RESCALE:
            e = launch_k(ctx->lev, last, k_moments_comb<MOM_COMB_RESCALE>, grid, block,
                         ctx->stream, a, ta);
            break;
        default:
            break;
    }
    if (e != hipSuccess || last) return e;
    return launch_strad<false>(ctx, a);
}

hipError_t launch_moments(wnnc_ctx_s *ctx, MomMode mode, const MomArgs &args) {
    MomArgs a = args;
    a.scalar = mode == MOM_SCALAR_SORTED || mode == MOM_SCALAR_CALLER || mode == MOM_CONST_HALF;
    if (a.order > 0 && a.momhi) return launch_moments_t<true>(ctx, mode, a);
    return launch_moments_t<false>(ctx, mode, a);
}

}  // namespace wnnc
