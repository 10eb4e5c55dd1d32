// Treecode traversal (Sec. 4.5, Alg. 4) for the three operators.
//
// A wavefront takes one task: 64 * TPL Morton-consecutive targets of one
// cloud (TPL groups of 64, one target per lane in each group), and walks the
// pre-order node range of that cloud once.  Every lane keeps its own Alg. 4
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
//
// HI (an extension of Alg. 4, for precision control): the representative
// term of an accepted node holding more than one point is followed by the
// order-1 (and, at order 2, order-2) terms of the Taylor expansion of the
// pair term about x_B, from the node's far-field moments.
#include <float.h>

#include "common.h"
#include "epilogue.h"
#include "internal.h"
#include "wave.h"

namespace wnnc {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
#define WNNC_AS4 __attribute__((address_space(4)))

// Loads through the constant address space: uniform addresses become SMEM
// loads (the arrays are not written during the kernel).
__device__ inline int4 ldc_i4(const int4 *p) {
    v4i v = *(const WNNC_AS4 v4i *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ inline float4 ldc_f4(const float4 *p) {
    v4f v = *(const WNNC_AS4 v4f *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ inline float ldc_f(const float *p) { return *(const WNNC_AS4 float *)p; }
__device__ inline int ldc_i(const int *p) { return *(const WNNC_AS4 int *)p; }

// The 64-byte record of a node: one 16-dword scalar load at a 32-bit byte
// offset from the base (the address needs one shift).
__device__ inline v16f ld_rec(const float4 *base, int node) {
    const WNNC_AS4 char *b = (const WNNC_AS4 char *)base;
    return *(const WNNC_AS4 v16f *)(b + ((unsigned)node << 6));
}

// The same load, issued without waiting for it: the compiler neither sinks
// it to its first use nor waits for it there.  rec_wait must come before
// any read of the result.
__device__ inline v16f rec_issue(const float4 *base, int node) {
    v16f r;
    const unsigned off = (unsigned)node << 6;
    asm volatile("s_load_dwordx16 %0, %1, %2" : "=s"(r) : "s"(base), "s"(off));
    return r;
}
// Waits for every scalar load in flight (they may complete out of order).
// The record is an operand, so that no read of it moves above the wait.
__device__ inline void rec_wait(v16f &r) { asm volatile("s_waitcnt lgkmcnt(0)" : "+s"(r)); }


// Deferred subtrees (TPL = 1, plain walk, Alg. 4's far field): at most
// kDeferEntries subtrees and kDeferTasks (subtree, target) tasks are held
// per wavefront before they are walked.
constexpr int kDeferEntries = 64;
constexpr int kDeferTasks = 1024;
// The packed walks hand out new tasks when more than kDeferSlack lanes
// have finished theirs.
constexpr int kDeferSlack = 24;

// Pair term without the 1/(4 pi) factor.  d = target - source, r2 = |d|^2.
//   A  : -(d . nu) / r^3
//   A^T: nu d / r^3                      (nu scalar, in v.x)
//   G  : nu / r^3 - 3 (d . nu) d / r^5
//   P  : g (m / r^3 - 3 (d . m) d / r^5) (g scalar in v.x; m = tv, the
//        target's own vector: the position-gradient walk)
//   T  : (3 r^2 (b (d . a) + a (d . b) + d (a . b)) - 15 d (d . a)(d . b)) / r^7
//        (a = v, b = tv: the third derivative of Phi contracted with the
//        source's and the target's vectors)
// `take` is false for lanes whose pair does not count: not selected by the
// traversal, or cut off (r < w, Sec. 4.4).  Their term is an exact zero, so
// that the unconditional add below leaves the sum unchanged.  The term is
// formed in FP32 and added to an FP64 per-target sum (FP64 adds issue at the
// FP32 rate on this chip), so the sum's rounding does not grow with the
// number of terms.
template <int OP>
__device__ inline void pair_term(float dx, float dy, float dz, float r2, float4 v,
                                 const float4 &tv, bool take, double &s, double &gx, double &gy,
                                 double &gz) {
    const float ri = __builtin_amdgcn_rsqf(r2);  // about 1 ulp
    const float ri2 = ri * ri;
    const float ri3 = ri2 * ri;
    if (OP == OP_A) {
        const float dm = fmaf(dx, v.x, fmaf(dy, v.y, dz * v.z));
        const float m3 = take ? -ri3 : 0.0f;
        s += (double)(dm * m3);
    } else if (OP == OP_T) {
        const float da = fmaf(dx, v.x, fmaf(dy, v.y, dz * v.z));
        const float db = fmaf(dx, tv.x, fmaf(dy, tv.y, dz * tv.z));
        const float ab = fmaf(v.x, tv.x, fmaf(v.y, tv.y, v.z * tv.z));
        // masked on r^2 as in G: rsq(inf) = 0 zeroes both factors
        const float ti = __builtin_amdgcn_rsqf(take ? r2 : __builtin_huge_valf());
        const float ti2 = ti * ti, ti5 = (ti2 * ti) * ti2;
        const float r5 = 3.0f * ti5;         // 3 / r^5
        const float r7 = 15.0f * ti5 * ti2;  // 15 / r^7
        const float q = r7 * da * db;
        gx += (double)fmaf(r5, fmaf(tv.x, da, fmaf(v.x, db, dx * ab)), -q * dx);
        gy += (double)fmaf(r5, fmaf(tv.y, da, fmaf(v.y, db, dy * ab)), -q * dy);
        gz += (double)fmaf(r5, fmaf(tv.z, da, fmaf(v.z, db, dz * ab)), -q * dz);
    } else if (OP == OP_P) {
        const float dm = fmaf(dx, tv.x, fmaf(dy, tv.y, dz * tv.z));
        // masked on r^2 as in G: rsq(inf) = 0 zeroes both factors (also at
        // r = 0, the target's own point)
        const float qi = __builtin_amdgcn_rsqf(take ? r2 : __builtin_huge_valf());
        const float qi2 = qi * qi, qi3 = qi2 * qi;
        const float a3 = v.x * qi3;
        const float b5 = v.x * (qi3 * qi2);
        const float c5 = 3.0f * dm * b5;
        gx += (double)fmaf(tv.x, a3, -c5 * dx);
        gy += (double)fmaf(tv.y, a3, -c5 * dy);
        gz += (double)fmaf(tv.z, a3, -c5 * dz);
    } else if (OP == OP_AT) {
        const float f = take ? v.x * ri3 : 0.0f;
        gx += (double)(f * dx);
        gy += (double)(f * dy);
        gz += (double)(f * dz);
    } else {
        const float dm = fmaf(dx, v.x, fmaf(dy, v.y, dz * v.z));
        // the mask goes on r^2 (one select instead of one per factor): a
        // lane that does not take the pair gets rsq(inf) = 0, so both
        // factors are exact zeros (also at r = 0); taken lanes compute
        // exactly what they would from r^2 itself
        const float gi = __builtin_amdgcn_rsqf(take ? r2 : __builtin_huge_valf());
        const float gi2 = gi * gi;
        const float a3 = gi2 * gi;
        const float b5 = a3 * gi2;
        const float c5 = 3.0f * dm * b5;
        gx += (double)fmaf(v.x, a3, -c5 * dx);
        gy += (double)fmaf(v.y, a3, -c5 * dy);
        gz += (double)fmaf(v.z, a3, -c5 * dz);
    }
}

// The same terms of A, A^T and G added to FP32 running sums of the
// lockstep walk (p0 for A; p0, p1, p2 for the vector operators).  The walk
// adds the running sums to its FP64 per-target sums whenever it changes
// depth (a descent, or the end of a subtree) and after the direct sum of a
// leaf's points, so a running sum holds the terms of at most 8 sibling
// nodes and of the points of at most one leaf, and carries a rounding error
// of at most about 2^-24 times their number times the sum of their
// magnitudes.  The last operation of each term is fused into the running
// sum.

template <int OP>
__device__ inline void pair_term_run(float dx, float dy, float dz, float r2, float4 v, bool take,
                                     float &p0, float &p1, float &p2) {
    if (OP == OP_A) {
        const float ri = __builtin_amdgcn_rsqf(r2);
        const float ri3 = (ri * ri) * ri;
        const float dm = fmaf(dx, v.x, fmaf(dy, v.y, dz * v.z));
        p0 = fmaf(dm, take ? -ri3 : 0.0f, p0);
    } else if (OP == OP_AT) {
        const float ri = __builtin_amdgcn_rsqf(r2);
        const float ri3 = (ri * ri) * ri;
        const float f = take ? v.x * ri3 : 0.0f;
        p0 = fmaf(f, dx, p0);
        p1 = fmaf(f, dy, p1);
        p2 = fmaf(f, dz, p2);
    } else {  // G, masked on r^2 as in pair_term: (nu - 3 (d . nu) d / r^2) / r^3
        const float dm = fmaf(dx, v.x, fmaf(dy, v.y, dz * v.z));
        const float gi = __builtin_amdgcn_rsqf(take ? r2 : __builtin_huge_valf());
        const float gi2 = gi * gi;
        const float a3 = gi2 * gi;
        const float u = (3.0f * dm) * gi2;
        p0 = fmaf(a3, fmaf(-u, dx, v.x), p0);
        p1 = fmaf(a3, fmaf(-u, dy, v.y), p1);
        p2 = fmaf(a3, fmaf(-u, dz, v.z), p2);
    }
}

typedef float v8f __attribute__((ext_vector_type(8)));

// Higher-order far-field terms (without the 1/(4 pi) factor) for target
// offset y = x - x_B = r u (|u| = 1), from the node's symmetric moments H
// (layout kHiStride; uniform across the wavefront).  With the derivatives
// of 1/r, each symmetric in all its indices,
//   T2_ij  = (3 y_i y_j - r^2 d_ij) / r^5
//   T3_ijk = (3 r^2 (d_ij y_k + d_ik y_j + d_jk y_i) - 15 y_i y_j y_k) / r^7
//   T4     = (105 yyyy - 15 r^2 (six d yy terms) + 3 r^4 (three d d terms)) / r^9
// the terms added to the representative term are, written in u so that no
// power of 1/r beyond the fifth is formed,
//   A  : - T2 : D + 1/2 T3 : Q   = (tr D - 3 u.D.u) / r^3 + (9 u.e - 15 q3) / (2 r^4)
//   A^T: T2 p - 1/2 T3 : q       = (3 u (u.p) - p) / r^3
//                                  - (3 (2 q u + u tr q) - 15 u (u.q.u)) / (2 r^4)
//   G  : T3 : D - 1/2 T4 : Q     = (3 (2 D u + u tr D) - 15 u (u.D.u)) / r^4
//                                  - (105 u q3 - 45 (a + u (u.e)) + 9 e) / (2 r^5)
// with a_m = sum_(k,n) u_k u_n Q_(m,k,n) and q3 = u.a.  The order-2 part is
// skipped at order 1.  `take` as in pair_term (a lane that does not take
// gets u = 0 and 1/r = 0: an exact 0).
template <int OP>
__device__ inline void far_terms(float dx, float dy, float dz, float r2, const v16f &H0,
                                 const v8f &H1, bool order2, bool take, double &s, double &gx,
                                 double &gy, double &gz) {
    const float ri = take ? __builtin_amdgcn_rsqf(r2) : 0.0f;
    const float u0 = dx * ri, u1 = dy * ri, u2 = dz * ri;
    const float ri2 = ri * ri;
    const float ri3 = ri2 * ri;
    const float ri4 = ri2 * ri2;
    auto h = [&](int i) -> float { return i < 16 ? H0[i] : H1[i - 16]; };
    if (OP == OP_AT) {
        // p_k = h(k); q pairs (00 01 02 11 12 22) = h(3..8); tr q = h(9)
        const float up = fmaf(u0, h(0), fmaf(u1, h(1), u2 * h(2)));
        float t0 = fmaf(3.0f * up, u0, -h(0)) * ri3;
        float t1 = fmaf(3.0f * up, u1, -h(1)) * ri3;
        float t2 = fmaf(3.0f * up, u2, -h(2)) * ri3;
        if (order2) {
            const float qu0 = fmaf(h(3), u0, fmaf(h(4), u1, h(5) * u2));
            const float qu1 = fmaf(h(4), u0, fmaf(h(6), u1, h(7) * u2));
            const float qu2 = fmaf(h(5), u0, fmaf(h(7), u1, h(8) * u2));
            const float uqu = fmaf(u0, qu0, fmaf(u1, qu1, u2 * qu2));
            const float trq = h(9), c = -7.5f * uqu;
            t0 -= fmaf(1.5f, fmaf(2.0f, qu0, u0 * trq), c * u0) * ri4;
            t1 -= fmaf(1.5f, fmaf(2.0f, qu1, u1 * trq), c * u1) * ri4;
            t2 -= fmaf(1.5f, fmaf(2.0f, qu2, u2 * trq), c * u2) * ri4;
        }
        gx += (double)t0;
        gy += (double)t1;
        gz += (double)t2;
        return;
    }
    // D pairs (00 01 02 11 12 22) = h(0..5), tr D = h(6)
    const float Du0 = fmaf(h(0), u0, fmaf(h(1), u1, h(2) * u2));
    const float Du1 = fmaf(h(1), u0, fmaf(h(3), u1, h(4) * u2));
    const float Du2 = fmaf(h(2), u0, fmaf(h(4), u1, h(5) * u2));
    const float uDu = fmaf(u0, Du0, fmaf(u1, Du1, u2 * Du2));
    const float trD = h(6);
    // Q triples (000 001 002 011 012 022 111 112 122 222) = h(7..16),
    // e = h(17..19)
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, q3 = 0.f, ue = 0.f;
    if (order2) {
        const float s00 = u0 * u0, s01 = 2.0f * u0 * u1, s02 = 2.0f * u0 * u2, s11 = u1 * u1,
                    s12 = 2.0f * u1 * u2, s22 = u2 * u2;
        a0 = fmaf(s00, h(7), fmaf(s01, h(8), fmaf(s02, h(9), fmaf(s11, h(10),
             fmaf(s12, h(11), s22 * h(12))))));
        a1 = fmaf(s00, h(8), fmaf(s01, h(10), fmaf(s02, h(11), fmaf(s11, h(13),
             fmaf(s12, h(14), s22 * h(15))))));
        a2 = fmaf(s00, h(9), fmaf(s01, h(11), fmaf(s02, h(12), fmaf(s11, h(14),
             fmaf(s12, h(15), s22 * h(16))))));
        q3 = fmaf(u0, a0, fmaf(u1, a1, u2 * a2));
        ue = fmaf(u0, h(17), fmaf(u1, h(18), u2 * h(19)));
    }
    if (OP == OP_A) {
        float t = fmaf(-3.0f, uDu, trD) * ri3;
        if (order2) t += fmaf(4.5f, ue, -7.5f * q3) * ri4;
        s += (double)t;
        return;
    }
    // G
    const float ri5 = ri4 * ri;
    const float c15 = -15.0f * uDu;
    float t0 = fmaf(3.0f, fmaf(2.0f, Du0, u0 * trD), c15 * u0) * ri4;
    float t1 = fmaf(3.0f, fmaf(2.0f, Du1, u1 * trD), c15 * u1) * ri4;
    float t2 = fmaf(3.0f, fmaf(2.0f, Du2, u2 * trD), c15 * u2) * ri4;
    if (order2) {
        const float c105 = 105.0f * q3;
        t0 -= 0.5f * fmaf(c105, u0, fmaf(-45.0f, fmaf(u0, ue, a0), 9.0f * h(17))) * ri5;
        t1 -= 0.5f * fmaf(c105, u1, fmaf(-45.0f, fmaf(u1, ue, a1), 9.0f * h(18))) * ri5;
        t2 -= 0.5f * fmaf(c105, u2, fmaf(-45.0f, fmaf(u2, ue, a2), 9.0f * h(19))) * ri5;
    }
    gx += (double)t0;
    gy += (double)t1;
    gz += (double)t2;
}

// The calling lane's bit of a wave-uniform lane mask (the mask is used as a
// condition directly, with no per-lane shift).
__device__ inline bool lane_in(unsigned long long mask) {
    return __builtin_amdgcn_inverse_ballot_w64(mask);
}


__device__ inline unsigned long long read_mask(uint32_t lo, uint32_t hi, int depth) {
    return (unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)lo, depth) |
           ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)hi, depth) << 32);
}

// One wavefront per task: TPL groups of 64 consecutive sorted targets
// (group k holds targets first + 64k + lane) walk the pre-order node range
// [first node, end node) of their cloud together.  Each group keeps its own
// mask stack and Alg. 4 decisions; the groups share the node loads and the
// control.
//
// A task whose range starts below the cloud's root is one part of a walk
// split for load balance (TPL = 1 only): the lanes' decisions at the
// ancestors of its first node are evaluated again (without their terms) to
// rebuild the mask stack, so the part makes exactly the decisions, and adds
// exactly the terms, that the whole walk makes over that node range.  The
// part's FP64 sums go to its part slot; k_combine adds the parts in order.
//
// PF: software pipelining of the node walk.  A node's successor is its skip
// pointer (subtree done) or the next node (descend); the skip successor's
// record is loaded while the node is visited, so that load overlaps the
// work on the node.
template <int OP, int MODE, bool COUNT, int TPL, bool PF, bool HI>
__global__ __launch_bounds__(kTravBlock) void k_traverse(TravArgs a) {
    const int lane = threadIdx.x & (kWave - 1);
    // the wavefront index is uniform; say so, so that the node walk below is
    // a scalar loop with scalar loads
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous range of tasks (Morton-ordered targets) so its L2 sees one
    // region of the tree.  Within an XCD, the workgroups of a block of
    // kCuBlock go round-robin to its 32 CUs as well: workgroup j of a block
    // takes task (j % 32) * (kCuBlock / 32) + j / 32, so that the tasks one
    // CU runs are neighbours and share more of the tree in its scalar cache
    // (a tail shorter than a block keeps the plain order; the far-field walk,
    // with its larger register footprint, is faster without it).
    constexpr int kCuBlock = 2048, kXcdCus = 32;
    const int G = gridDim.x, b = blockIdx.x;
    const int q = G >> 3, r = G & 7, x = b & 7;
    int L = b >> 3;
    if (!HI && L < (q + (x < r ? 1 : 0)) / kCuBlock * kCuBlock) {
        const int j = L % kCuBlock;
        L += (j % kXcdCus) * (kCuBlock / kXcdCus) + j / kXcdCus - j;
    }
    const int lb = x * q + (x < r ? x : r) + L;
    const int wave = lb * (kTravBlock / kWave) + wv;
    if (wave >= a.ntasks) return;
    const int4 task = ldc_i4(a.tasks + wave);
    const int first = task.x, last = task.y, nbeg = task.z, nend = task.w;
    const int tslot = ldc_i(a.task_slot + wave);

    float tx[TPL], ty[TPL], tz[TPL];
    float4 tv[TPL];  // P: the target's own vector (unused by the other operators)
    double s[TPL], gx[TPL], gy[TPL], gz[TPL];
    bool valid[TPL];
    uint32_t mlo[TPL], mhi[TPL];
    // the mask of the depth visited last (equal to its stack entry), so that
    // a visit at the same depth (a sibling, or a child after a descent)
    // needs no read of the stack
    unsigned long long cur[TPL];
    int cur_depth = -1;
    // FP32 running sums of the lockstep walk (A, A^T, G)
    constexpr bool RUNS = OP == OP_A || OP == OP_AT || OP == OP_G;
    float run0[TPL], run1[TPL], run2[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) run0[k] = run1[k] = run2[k] = 0.0f;
    auto add_runs = [&]() {
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            if (OP == OP_A) {
                s[k] += (double)run0[k];
            } else {
                gx[k] += (double)run0[k];
                gy[k] += (double)run1[k];
                gz[k] += (double)run2[k];
            }
            run0[k] = run1[k] = run2[k] = 0.0f;
        }
    };
    uint32_t cnt = 0;
    int visits = 0;
    // Deferred subtrees: a subtree that at most a.defer_k lanes of the group
    // need is not walked in lockstep; its (first node, end node) goes to
    // dent and one (entry, lane) task per such lane to dtask.  flush() then
    // walks the tasks packed across the lanes, each lane walking one
    // target's subtree on its own (vector record loads), and adds each
    // task's FP64 sums to its target's slot of dacc.  The decisions and
    // terms are those of the lockstep walk; only the order of the FP64
    // additions differs.
    constexpr bool DEFER = TPL == 1 && !PF && !HI && MODE != TR_PLAN;
    __shared__ int2 dent[DEFER ? kDeferEntries : 1];
    __shared__ uint16_t dtask[DEFER ? kDeferTasks : 1];
    __shared__ double dacc[DEFER ? 3 : 1][DEFER ? kWave : 1];
    __shared__ float4 dtgt[DEFER ? kWave : 1];
    __shared__ float4 dtv[DEFER && (OP == OP_P || OP == OP_T) ? kWave : 1];
    int dne = 0, dnt = 0;  // entries and tasks held (wave-uniform)
    uint32_t dcnt = 0;     // pairs of this lane's deferred steps (COUNT)
    if constexpr (DEFER) {
        dacc[0][lane] = 0.0;
        dacc[1][lane] = 0.0;
        dacc[2][lane] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = first + k * kWave + lane;
        valid[k] = t < last;
        tx[k] = ty[k] = tz[k] = 0.f;
        tv[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        if ((OP == OP_P || OP == OP_T) && valid[k]) tv[k] = a.tvec[t];
        if (valid[k]) {
            const float4 p = a.tpts[t];
            tx[k] = p.x, ty[k] = p.y, tz[k] = p.z;
        }
        s[k] = gx[k] = gy[k] = gz[k] = 0.0;
        // mask stack: lane d holds the mask of group-k lanes inside at depth d
        const unsigned long long act0 = __ballot(valid[k]);
        mlo[k] = lane == 0 ? (uint32_t)act0 : 0u;
        mhi[k] = lane == 0 ? (uint32_t)(act0 >> 32) : 0u;
    }

    // A part of a split walk (task slot < 0): the decisions at the ancestors
    // of its first node, from the cloud's root down.  The ancestors are
    // listed with the tasks (one 64-byte load), so their records do not
    // wait for each other.  A whole walk starts at the root and has none.
    if (TPL == 1 && tslot < 0) {  // (walks are split only with one group per wavefront)
        typedef int v16i __attribute__((ext_vector_type(16)));
        const v16i C = *(const WNNC_AS4 v16i *)(a.chain + (int64_t)wave * kChainStride);
        const int na = C[0];
#pragma unroll
        for (int d = 0; d < kMaxDepth; ++d) {
            if (d >= na) continue;
            const v16f R = ld_rec(a.mom, C[1 + d]);
            const int depth = __float_as_int(R[3]) & 15;
#pragma unroll
            for (int k = 0; k < TPL; ++k) {
                // (a zero-weight node, threshold -1, is opened by no lane)
                const unsigned long long act = read_mask(mlo[k], mhi[k], depth);
                const float dx = (tx[k] - R[0]) - R[8], dy = (ty[k] - R[1]) - R[9],
                            dz = (tz[k] - R[2]) - R[10];
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const unsigned long long open = act & ~__ballot(r2 > R[11]);
                if (lane == depth + 1) {
                    mlo[k] = (uint32_t)open;
                    mhi[k] = (uint32_t)(open >> 32);
                }
            }
        }
    }

    // Walks the held tasks: every lane takes the next task whenever it has
    // none, so the lanes stay busy until the tasks run out.
    auto flush = [&]() {
      if constexpr (DEFER) {
        // each lane's target (and its vector), for the lanes that walk it
        dtgt[lane] = make_float4(tx[0], ty[0], tz[0], 0.f);
        if (OP == OP_P || OP == OP_T) dtv[lane] = tv[0];
        __syncthreads();  // the wavefront's LDS writes are visible
        const int nt = dnt;
        int nextt = 0;           // next task to hand out (wave-uniform)
        int node = 0, end = 0;   // this lane's walk
        int tg = -1;             // its target lane (-1: no task)
        float px = 0.f, py = 0.f, pz = 0.f;
        float4 ptv = make_float4(0.f, 0.f, 0.f, 0.f);
        double ps = 0.0, pgx = 0.0, pgy = 0.0, pgz = 0.0;
        for (;;) {
            const bool done = node >= end;
            if (done && tg >= 0) {  // the task ended: its sums to the target
                if (OP == OP_A) {
                    atomicAdd(&dacc[0][tg], ps);
                } else {
                    atomicAdd(&dacc[0][tg], pgx);
                    atomicAdd(&dacc[1][tg], pgy);
                    atomicAdd(&dacc[2][tg], pgz);
                }
                ps = pgx = pgy = pgz = 0.0;
                tg = -1;
            }
            const unsigned long long need = __ballot(done);
            const int my = nextt + (int)__builtin_amdgcn_mbcnt_hi(
                                       (uint32_t)(need >> 32),
                                       __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
            nextt += __popcll(need);
            if (done && my < nt) {
                const int tk = dtask[my];
                const int2 en = dent[tk >> 6];
                node = en.x;
                end = en.y;
                tg = tk & 63;
                const float4 p = dtgt[tg];
                px = p.x, py = p.y, pz = p.z;
                if (OP == OP_P || OP == OP_T) ptv = dtv[tg];
            }
            bool act = node < end;
            if (__ballot(act) == 0ull && nextt >= nt) break;
            // step the walks until more than kDeferSlack lanes are idle
            // while tasks remain (then hand out more), or until all are
            // done: the hand-out is not paid on every step
            const int keep = nextt < nt ? kWave - kDeferSlack : 1;
            do {
                if (act) {
                    // the whole record in one round of loads; the branches below
                    // are selects, except the rare direct sum of a leaf's points
                    const float4 *rb =
                        (const float4 *)((const char *)a.mom + ((uint32_t)node << 6));
                    const float4 R0 = rb[0], R1 = rb[1], R2 = rb[2];
                    const int fl = __float_as_int(R0.w);
                    const int sk = __float_as_int(R1.w);
                    const float dx = (px - R0.x) - R2.x, dy = (py - R0.y) - R2.y,
                                dz = (pz - R0.z) - R2.z;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    // accepted (a single-point leaf and a zero-weight node
                    // always are)
                    const bool far = r2 > R2.w;
                    // (a node of zero weight adds an exact zero and is not
                    // counted)
                    if (COUNT)
                        dcnt += (far && !(R2.w < 0.f && R1.x == 0.f && R1.y == 0.f &&
                                          R1.z == 0.f)) ? 1u : 0u;
                    pair_term<OP>(dx, dy, dz, r2, make_float4(R1.x, R1.y, R1.z, 0.f), ptv,
                                  far && r2 >= a.w2, ps, pgx, pgy, pgz);
                    const bool cell = !far && (fl & kRecLeaf) != 0;
                    if (cell) {  // the points of a depth-D cell (or a leaf of several)
                        const float4 R3 = rb[3];
                        const int jb = __float_as_int(R3.x), je = __float_as_int(R3.y);
                        for (int j = jb; j < je; ++j) {
                            const float4 Q = a.pts[j];
                            float4 S;
                            if (OP == OP_AT || OP == OP_P)
                                S = make_float4(a.srcs[j], 0.f, 0.f, 0.f);
                            else
                                S = a.src4[j];
                            const float ex = px - Q.x, ey = py - Q.y, ez = pz - Q.z;
                            const float e2 = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
                            if (COUNT) ++dcnt;
                            pair_term<OP>(ex, ey, ez, e2, S, ptv, e2 >= a.w2, ps, pgx, pgy, pgz);
                        }
                    }
                    node = (far || cell) ? sk : node + 1;
                }
                act = node < end;
            } while (__popcll(__ballot(act)) >= keep);
        }
        __syncthreads();  // every task's sums are in dacc
        dne = 0;
        dnt = 0;
      }
    };

    // One node visit for all groups; returns the next node in pre-order.
    auto visit = [&](const v16f &R, int node) -> int {
        if (MODE == TR_PLAN) {
            if (visits > 0 && visits % kPlanStep == 0 && visits / kPlanStep <= kPlanCap &&
                lane == 0)
                a.plan[(int64_t)tslot * kPlanStride + visits / kPlanStep] = node;
            ++visits;
        }
        const int flags = __float_as_int(R[3]);
        const int skip = __float_as_int(R[7]);
        const int depth = flags & 15;
        const float thr2 = R[11];  // -1 for a single-point leaf: always taken
        const float4 V = make_float4(R[4], R[5], R[6], 0.f);
        if (depth != cur_depth) {
            if constexpr (RUNS) add_runs();
#pragma unroll
            for (int k = 0; k < TPL; ++k) cur[k] = read_mask(mlo[k], mhi[k], depth);
            cur_depth = depth;
        }
        unsigned long long open[TPL];
        unsigned long long any = 0ull;
        // HI: the accepted lanes and their offsets, for the far-field terms;
        // the node's moments are loaded first, so that their latency
        // overlaps the representative terms
        unsigned long long htake[TPL];
        float hdx[TPL], hdy[TPL], hdz[TPL], hr2[TPL];
        v16f H0;
        v8f H1;
        const bool hi_node = HI && !(flags & kRecSingle);
        if (hi_node) {
            const WNNC_AS4 char *hb =
                (const WNNC_AS4 char *)a.momhi + (unsigned)node * (unsigned)(kHiStride * 4);
            H0 = *(const WNNC_AS4 v16f *)hb;
            H1 = *(const WNNC_AS4 v8f *)(hb + 64);
        }
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            // lanes of group k inside at this depth; of those, the ones that
            // accept the representative (far) and the ones that need B's
            // children (open), all as wave-uniform lane masks
            const unsigned long long act = cur[k];
            // (x - hi) is exact for a target near the node; then the low part
            const float dx = (tx[k] - R[0]) - R[8], dy = (ty[k] - R[1]) - R[9],
                        dz = (tz[k] - R[2]) - R[10];
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const unsigned long long far = act & __ballot(r2 > thr2);
            // w2 >= the smallest normal float, so the cutoff also drops r = 0
            // (and keeps denormal arguments away from the hardware rsq).
            const unsigned long long take = far & __ballot(r2 >= a.w2);
            if constexpr (RUNS)
                pair_term_run<OP>(dx, dy, dz, r2, V, lane_in(take), run0[k], run1[k], run2[k]);
            else
                pair_term<OP>(dx, dy, dz, r2, V, tv[k], lane_in(take), s[k], gx[k], gy[k], gz[k]);
            // (a node of zero weight, threshold -1 and nu_B = 0, adds an
            // exact zero and is not counted)
            if (COUNT && !(thr2 < 0.f && V.x == 0.f && V.y == 0.f && V.z == 0.f))
                cnt += (uint32_t)__popcll(far);
            open[k] = act & ~far;
            any |= open[k];
            if (HI) htake[k] = take, hdx[k] = dx, hdy[k] = dy, hdz[k] = dz, hr2[k] = r2;
        }
        if (hi_node) {
            unsigned long long anyt = 0ull;
#pragma unroll
            for (int k = 0; k < TPL; ++k) anyt |= htake[k];
            if (anyt != 0ull) {
#pragma unroll
                for (int k = 0; k < TPL; ++k)
                    far_terms<OP>(hdx[k], hdy[k], hdz[k], hr2[k], H0, H1, a.order >= 2,
                                  lane_in(htake[k]), s[k], gx[k], gy[k], gz[k]);
            }
        }
        if (any == 0ull) return skip;
        if (flags & kRecLeaf) {
            // several points in a depth-D cell: direct sum for the lanes
            // that did not accept the representative
            const int jb = __float_as_int(R[12]), je = __float_as_int(R[13]);
            for (int j = jb; j < je; ++j) {
                const float4 Q = ldc_f4(a.pts + j);
                float4 S;
                if (OP == OP_AT || OP == OP_P)
                    S = make_float4(ldc_f(a.srcs + j), 0.f, 0.f, 0.f);
                else
                    S = ldc_f4(a.src4 + j);
#pragma unroll
                for (int k = 0; k < TPL; ++k) {
                    const float ex = tx[k] - Q.x, ey = ty[k] - Q.y, ez = tz[k] - Q.z;
                    const float e2 = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
                    const unsigned long long take = open[k] & __ballot(e2 >= a.w2);
                    if constexpr (RUNS)
                        pair_term_run<OP>(ex, ey, ez, e2, S, lane_in(take), run0[k], run1[k],
                                          run2[k]);
                    else
                        pair_term<OP>(ex, ey, ez, e2, S, tv[k], lane_in(take), s[k], gx[k],
                                      gy[k], gz[k]);
                    if (COUNT) cnt += (uint32_t)__popcll(open[k]);
                }
                if constexpr (RUNS) add_runs();
            }
            return skip;
        }
        if (DEFER && a.defer_k > 0 && __popcll(open[0]) <= a.defer_k) {
            // defer the subtree for the few lanes that need it
            const unsigned long long dm = open[0];
            if constexpr (DEFER) {
            if (lane == 0) dent[dne] = make_int2(node + 1, min(skip, nend));
            if (lane_in(dm)) {
                const int pos = dnt + (int)__builtin_amdgcn_mbcnt_hi(
                                          (uint32_t)(dm >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)dm, 0u));
                dtask[pos] = (uint16_t)((dne << 6) | lane);
            }
            }
            dne += 1;
            dnt += __popcll(dm);
            if (dne == kDeferEntries || dnt > kDeferTasks - kWave) flush();
            return skip;
        }
        // push: lane depth + 1 takes the mask (selected by a scalar lane mask)
        if constexpr (RUNS) add_runs();
        const bool at = lane_in(1ull << (depth + 1));
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            mlo[k] = at ? (uint32_t)open[k] : mlo[k];
            mhi[k] = at ? (uint32_t)(open[k] >> 32) : mhi[k];
            cur[k] = open[k];
        }
        cur_depth = depth + 1;
        return node + 1;
    };

    // (with the far-field moments the walk keeps plain loads: their extra
    // scalar registers would crowd the record in flight)
    if (!PF || HI) {
        for (int node = nbeg; node < nend;) node = visit(ld_rec(a.mom, node), node);
        if (DEFER && dne > 0) flush();
    } else if (nbeg < nend) {
        // Software-pipelined walk.  A wait for a scalar load covers every
        // scalar load in flight, so the skip successor's record is issued
        // right after the wait for the current one and arrives while the
        // current node is visited; when the walk descends instead, the first
        // child is loaded then.  Loaded indices are clamped to the range,
        // and the walk advances by at least one node per visit.
        int node = nbeg;
        // the cutoff is read in every visit: have the compiler wait for its
        // load here, so that it places no wait (which would also wait for
        // the record in flight) inside the loop
        asm volatile("" ::"s"(a.w2));
        // two record buffers in turn, so that no record is copied
        v16f RA = rec_issue(a.mom, node), RB;
        rec_wait(RA);
        for (;;) {
            int sk = min(max(__float_as_int(RA[7]), node + 1), nend - 1);
            RB = rec_issue(a.mom, sk);
            int nx = max(visit(RA, node), node + 1);
            rec_wait(RB);
            if (nx >= nend) break;
            if (nx != sk) {
                RB = rec_issue(a.mom, nx);
                rec_wait(RB);
            }
            node = nx;
            sk = min(max(__float_as_int(RB[7]), node + 1), nend - 1);
            RA = rec_issue(a.mom, sk);
            nx = max(visit(RB, node), node + 1);
            rec_wait(RA);
            if (nx >= nend) break;
            if (nx != sk) {
                RA = rec_issue(a.mom, nx);
                rec_wait(RA);
            }
            node = nx;
        }
    }

    if constexpr (RUNS) add_runs();
    if constexpr (DEFER) {  // the deferred tasks' sums of each target (0 if none)
        if (OP == OP_A) {
            s[0] += dacc[0][lane];
        } else {
            gx[0] += dacc[0][lane];
            gy[0] += dacc[1][lane];
            gz[0] += dacc[2][lane];
        }
        if (COUNT) {
            uint32_t t = dcnt;
#pragma unroll
            for (int d = kWave / 2; d > 0; d >>= 1) t += __shfl_xor(t, d, kWave);
            cnt += t;
        }
    }
    if (COUNT) {  // cnt is wave-uniform: the pairs of all lanes
        if (lane == 0) atomicAdd(a.pairs + OP, (unsigned long long)cnt);
    }
    if (MODE == TR_PLAN) {
        if (lane == 0) a.plan[(int64_t)tslot * kPlanStride] = visits;
        return;
    }
    if (tslot < 0) {  // one part of a split walk (TPL = 1): its sums, rounded to FP32
        float *qp = a.parts + (int64_t)(-1 - tslot) * (3 * kWave);
        if (OP == OP_A) {
            qp[lane] = (float)s[0];
        } else {
            qp[lane] = (float)gx[0];
            qp[kWave + lane] = (float)gy[0];
            qp[2 * kWave + lane] = (float)gz[0];
        }
        return;
    }
    double e = 0.0, e2 = 0.0;
    unsigned nflip = 0;
    float4 nu;
#pragma unroll
    for (int k = 0; k < TPL; ++k)
        if (valid[k])
            finish_target<OP, MODE>(a, first + k * kWave + lane, s[k], gx[k], gy[k], gz[k], e, e2,
                                    nflip, nu);
    finish_group<MODE>(a, tslot, first, lane, e, e2, nflip);
}

// Groups walked in parts: one wavefront per group adds its parts' sums in
// part order (sum_parts) and runs the epilogue.
template <int OP, int MODE>
__global__ __launch_bounds__(kWave) void k_combine(TravArgs a, const int4 *__restrict__ groups,
                                                   const int32_t *__restrict__ gslot) {
    const int lane = threadIdx.x;
    const int4 g = ldc_i4(groups + blockIdx.x);
    double s = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    sum_parts<OP>(a.parts, g.z, g.w, lane, s, gx, gy, gz);
    double e = 0.0, e2 = 0.0;
    unsigned nflip = 0;
    const int t = g.x + lane;
    float4 nu;
    if (t < g.y) finish_target<OP, MODE>(a, t, s, gx, gy, gz, e, e2, nflip, nu);
    finish_group<MODE>(a, ldc_i(gslot + blockIdx.x), g.x, lane, e, e2, nflip);
}

int trav_blocks(int64_t ntasks) {
    return (int)((ntasks + kTravBlock / kWave - 1) / (kTravBlock / kWave));
}

template <int OP, int MODE, int TPL, bool HI>
static hipError_t launch_tpl_hi(wnnc_ctx_s *ctx, bool count, const TravArgs &a) {
    const dim3 grid((unsigned)trav_blocks(a.ntasks)), block(kTravBlock);
    auto &ev = ctx->lev;
    hipStream_t st = ctx->stream;
    if (a.prefetch)
        return count ? launch_k(ev, true, k_traverse<OP, MODE, true, TPL, true, HI>, grid, block, st, a)
                     : launch_k(ev, true, k_traverse<OP, MODE, false, TPL, true, HI>, grid, block, st, a);
    return count ? launch_k(ev, true, k_traverse<OP, MODE, true, TPL, false, HI>, grid, block, st, a)
                 : launch_k(ev, true, k_traverse<OP, MODE, false, TPL, false, HI>, grid, block, st, a);
}

template <int OP, int MODE, int TPL>
static hipError_t launch_tpl(wnnc_ctx_s *ctx, bool count, const TravArgs &a) {
    if constexpr (OP == OP_P || OP == OP_T) {
        // the position-gradient walk has the representative far field only
        return launch_tpl_hi<OP, MODE, TPL, false>(ctx, count, a);
    } else {
        if (a.order > 0 && a.momhi) return launch_tpl_hi<OP, MODE, TPL, true>(ctx, count, a);
        return launch_tpl_hi<OP, MODE, TPL, false>(ctx, count, a);
    }
}

template <int OP, int MODE>
static hipError_t launch_one(wnnc_ctx_s *ctx, bool count, const TravArgs &a) {
    if (a.ntasks <= 0) return hipSuccess;
    switch (a.tpl) {
        case 1: return launch_tpl<OP, MODE, 1>(ctx, count, a);
        case 2: return launch_tpl<OP, MODE, 2>(ctx, count, a);
        case 4: return launch_tpl<OP, MODE, 4>(ctx, count, a);
        default: return hipErrorInvalidValue;
    }
}

template <int OP, int MODE>
static hipError_t launch_comb(wnnc_ctx_s *ctx, const TravArgs &a) {
    if (a.ntasks <= 0 || ctx->nsplit <= 0) return hipSuccess;
    return launch_k(ctx->lev, true, k_combine<OP, MODE>, dim3((unsigned)ctx->nsplit), dim3(kWave),
                    ctx->stream, a, ctx->split_groups.p, ctx->split_slot.p);
}

hipError_t launch_traverse(wnnc_ctx_s *ctx, Op op, TravMode mode, bool count, const TravArgs &a) {
    if (op == OP_A) {
        if (mode == TR_OUT_CALLER) return launch_one<OP_A, TR_OUT_CALLER>(ctx, count, a);
        if (mode == TR_RHO) return launch_one<OP_A, TR_RHO>(ctx, count, a);
        if (mode == TR_TSUM) return launch_one<OP_A, TR_TSUM>(ctx, count, a);
        if (mode == TR_SCALE) return launch_one<OP_A, TR_SCALE>(ctx, count, a);
    } else if (op == OP_AT) {
        if (mode == TR_OUT_CALLER) return launch_one<OP_AT, TR_OUT_CALLER>(ctx, count, a);
        if (mode == TR_R) return launch_one<OP_AT, TR_R>(ctx, count, a);
    } else if (op == OP_G) {
        if (mode == TR_OUT_CALLER) return launch_one<OP_G, TR_OUT_CALLER>(ctx, count, a);
        if (mode == TR_RESCALE) return launch_one<OP_G, TR_RESCALE>(ctx, count, a);
    } else if (op == OP_P) {
        if (mode == TR_POSGRAD) return launch_one<OP_P, TR_POSGRAD>(ctx, count, a);
    } else {
        if (mode == TR_OUT_CALLER) return launch_one<OP_T, TR_OUT_CALLER>(ctx, count, a);
        if (mode == TR_ACCUM) return launch_one<OP_T, TR_ACCUM>(ctx, count, a);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_combine(wnnc_ctx_s *ctx, Op op, TravMode mode, const TravArgs &a) {
    if (op == OP_A) {
        if (mode == TR_OUT_CALLER) return launch_comb<OP_A, TR_OUT_CALLER>(ctx, a);
        if (mode == TR_RHO) return launch_comb<OP_A, TR_RHO>(ctx, a);
        if (mode == TR_TSUM) return launch_comb<OP_A, TR_TSUM>(ctx, a);
        if (mode == TR_SCALE) return launch_comb<OP_A, TR_SCALE>(ctx, a);
    } else if (op == OP_AT) {
        if (mode == TR_OUT_CALLER) return launch_comb<OP_AT, TR_OUT_CALLER>(ctx, a);
        if (mode == TR_R) return launch_comb<OP_AT, TR_R>(ctx, a);
    } else if (op == OP_G) {
        if (mode == TR_OUT_CALLER) return launch_comb<OP_G, TR_OUT_CALLER>(ctx, a);
        if (mode == TR_RESCALE) return launch_comb<OP_G, TR_RESCALE>(ctx, a);
    } else if (op == OP_P) {
        if (mode == TR_POSGRAD) return launch_comb<OP_P, TR_POSGRAD>(ctx, a);
    } else {
        if (mode == TR_OUT_CALLER) return launch_comb<OP_T, TR_OUT_CALLER>(ctx, a);
        if (mode == TR_ACCUM) return launch_comb<OP_T, TR_ACCUM>(ctx, a);
    }
    return hipErrorInvalidValue;
}

hipError_t record_plan(wnnc_ctx_s *ctx, const TravArgs &a) {
    if (a.ntasks <= 0) return hipSuccess;
    if (a.tpl != 1 || ctx->nsplit != 0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)trav_blocks(a.ntasks)), block(kTravBlock);
    hipLaunchKernelGGL((k_traverse<OP_AT, TR_PLAN, false, 1, false, false>), grid, block, 0,
                       ctx->stream, a);
    return hipGetLastError();
}

}  // namespace wnnc
