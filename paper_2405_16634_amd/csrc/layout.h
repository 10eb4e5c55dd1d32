// Data layout and kernel arguments shared by the device code: constants,
// the node topology and node record formats, operator and epilogue modes,
// and the argument blocks of the moment and traversal kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wnnc.h"

namespace wnnc {

constexpr int kWave = 64;
constexpr int kChunk = 512;      // points per moment-pass chunk (one workgroup)
constexpr int kTravBlock = 64;  // traversal workgroup: one wave (finest dispatch)
constexpr int kMaxDepth = 15;    // 15 levels below the root: 45-bit Morton keys

// Node topology, one int4 per node in depth-first pre-order:
//   x = skip: index of the first node after this node's subtree
//   y = begin, z = end: the node's points are sorted positions [begin, end)
//   w = depth | (leaf << 4)
// The first child of an internal node is the next node (index + 1).
__host__ __device__ inline int topo_depth(int meta) { return meta & 15; }
__host__ __device__ inline int topo_leaf(int meta) { return (meta >> 4) & 1; }

// Node record read by the traversal, 64 bytes per node (one 16-dword scalar
// load).  The moment pass writes hi(x_B), nu_B and part [2]; the flags, the
// skip pointer and part [3] are written once, with the tree (of a
// single-point leaf, whose representative is its point, the moment pass
// writes only nu_B: its position and threshold are written with the tree):
//   [0] hi(x_B).x, .y, .z, flags (int bits)
//   [1] nu_B (3 floats; a scalar attribute in .x), skip (int bits)
//   [2] lo(x_B).x, .y, .z, (c * width)^2 (the acceptance threshold)
//   [3] first point, end point (int bits), 0, 0
// with x_B = hi + lo to about 2^-48 (hi = FP32 rounding of the FP64 x_B,
// lo = FP32 rounding of the rest), so that target - x_B keeps full FP32
// precision when the target is close to the node.
// flags = depth | leaf << 4 | single-point leaf << 5.  A node of zero
// weight (every attribute in it zero) has threshold -1 and nu_B = 0: every
// target takes it as an exact zero term, and none descends into it.
// The traversal addresses records with 32-bit byte offsets: at most
// kMaxNodes nodes.
constexpr int kRecStride = 4;
// Far-field moments about x_B of every node (orders 1 and 2 of the far
// field), kHiStride floats per node.  The Taylor terms contract them with
// derivatives of 1/r, which are symmetric in all their indices, so only the
// symmetric parts are kept (d_j = x_j - x_B):
//   vector nu: [0..5]   D_(k,n)   = sym of sum_j d_jk nu_jn, pairs
//                                   (0,0) (0,1) (0,2) (1,1) (1,2) (2,2)
//              [6]      tr D      = sum_j d_j . nu_j
//              [7..16]  Q_(k,n,l) = sym of sum_j d_jk d_jn nu_jl, triples
//                                   000 001 002 011 012 022 111 112 122 222
//              [17..19] e_m       = sum_k Q_(k,k,m)
//   scalar rho: [0..2]  p_k       = sum_j rho_j d_jk
//              [3..8]   q_(k,n)   = sum_j rho_j d_jk d_jn, pairs as above
//              [9]      tr q
constexpr int kHiStride = 24;
// FP64 partial sums per chunk and per straddler in the moment pass: 7 for
// the representatives, 16 more with the raw (about the origin) symmetric
// far-field moments.
constexpr int kMomSlots = 24;
constexpr int kMomBase = 7;
constexpr int kMomHi = kMomBase + 16;
constexpr int64_t kMaxNodes = int64_t(1) << 26;
constexpr int kRecLeaf = 16;
constexpr int kRecSingle = 32;
// The moment pass's view of a node started inside a chunk, one int2 per
// node: (first point, end point | depth << kMnodeEndBits) for a node that
// ends inside the chunk it starts in, (first point, -1 - straddler slot)
// for one that does not.
constexpr int kMnodeEndBits = 26;
constexpr int kMnodeEndMask = (1 << kMnodeEndBits) - 1;
static_assert(kMaxNodes <= (int64_t(1) << kMnodeEndBits), "end points fit the node view");

enum Op { OP_A = WNNC_OP_A, OP_AT = WNNC_OP_AT, OP_G = WNNC_OP_G, OP_P = WNNC_OP_P, OP_T = WNNC_OP_T };
constexpr int kOpKinds = 5;

// Warm-start MLP: 48 -> 64 -> 64 -> 3; flat FP32 parameter vector, row-major
// [in][out] weights each followed by its bias.
constexpr int kMlpIn = 48, kMlpHidden = 64, kMlpOut = 3;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpIn * kMlpHidden;
constexpr int kOffW2 = kOffB1 + kMlpHidden;
constexpr int kOffB2 = kOffW2 + kMlpHidden * kMlpHidden;
constexpr int kOffW3 = kOffB2 + kMlpHidden;
constexpr int kOffB3 = kOffW3 + kMlpHidden * kMlpOut;
constexpr int kMlpParams = kOffB3 + kMlpOut;  // 7491
static_assert(kMlpParams == WNNC_MLP_PARAMS, "parameter count");

// Moment-pass input modes.
enum MomMode {
    MOM_VEC_SORTED = 0,    // nu = src4[i] (sorted float4)
    MOM_SCALAR_SORTED = 1, // nu = srcs[i] (sorted float)
    MOM_VEC_CALLER = 2,    // nu = n[perm[i]] * (sigma ? sigma[perm[i]] : 1); writes out4[i]
    MOM_SCALAR_CALLER = 3, // nu = s[perm[i]]; writes outs[i]
    MOM_AXPY = 4,          // nu = src4[i] + alpha * r4[i]; writes out4[i]
    MOM_CONST_HALF = 5,    // nu = 1/2 (scalar); writes outs[i]
    // nu = the output of the walk just launched without its combining pass:
    // the pass first runs that pass's epilogue for the split groups (its
    // parts summed in order), 64-point groups aligned with its wavefronts
    MOM_COMB_RHO = 6,      // A walk, TR_RHO: nu = rho (scalar)
    MOM_COMB_R = 7,        // A^T walk, TR_R: nu = r
    MOM_COMB_RESCALE = 8,  // G walk, TR_RESCALE: nu = the updated mu
};

// Key layout: the cloud index sits above the 45 Morton bits, so one sort
// groups the points cloud by cloud and each cloud gets its own root.
constexpr int kMortonBits = 45;

// Traversal epilogues.
enum TravMode {
    TR_OUT_CALLER = 0,  // write the operator value to caller order (API calls)
    TR_RHO = 1,         // A: rho = 1/2 - s (sorted), block partial of rho^2
    TR_R = 2,           // A^T: r (sorted float4), block partial of |r|^2
    TR_TSUM = 3,        // A: block partial of s^2 only
    TR_RESCALE = 4,     // G: mu <- G |mu| / |G| (sorted float4)
    TR_SCALE = 5,       // A: block partials of s and s^2 (warm-start scale)
    TR_PLAN = 6,        // no output: record the walk of each group (split planning)
    TR_POSGRAD = 7,     // P: out = p / (4 pi) + g grad F, caller order (position gradient)
    TR_ACCUM = 8,       // out = sum / (4 pi) + base, caller order (base in gradf)
};

// Split planning: the walk of every 64-target group is recorded as its node
// visit count and the node at every kPlanStep-th visit (up to kPlanCap of
// them), kPlanStride ints per group.
constexpr int kPlanStep = 64;
constexpr int kPlanCap = 63;
constexpr int kPlanStride = kPlanCap + 1;

// Per task, the ancestors of its first node (a part of a split walk):
// their count, then the nodes from the cloud's root down (at most one per
// depth above the deepest), kChainStride ints per task.
constexpr int kChainStride = kMaxDepth + 1;

struct MomArgs {
    const float4 *pts;       // sorted points
    const int2 *mnode;       // per node: the moment pass's view (kMnodeEndBits)
    const uint32_t *node_off;
    const uint32_t *tail_off;
    const int2 *tail_list;   // (straddler slot, end point) of the straddlers ending in each chunk
    const int32_t *strad_node;
    const int4 *strad_topo;  // topology of each straddler
    const uint32_t *perm;
    const float4 *src4;      // sorted vector input
    const float *srcs;       // sorted scalar input
    const float4 *r4;        // axpy direction
    const double *alpha;     // axpy step per cloud (device)
    const int32_t *cloud;    // cloud index per sorted point (batched axpy)
    const float *cn;         // caller-order (N,3) input
    const float *csig;       // caller-order sigma (may be null)
    const float *cs;         // caller-order scalar input
    float4 *out4;
    float *outs;
    double *chunk_tot;       // kMomSlots doubles per chunk, slot-major
    double *head;            // kMomSlots doubles per straddler
    double *tail;            // kMomSlots doubles per straddler
    float4 *mom;             // node records, kRecStride float4 per node
    float *momhi;            // far-field moments, kHiStride floats per node (order >= 1)
    float *wout;             // optional: W = sum |nu| per node (inspection)
    float thr2[16];          // squared acceptance distance per depth d, into records
    int n;
    int n_strad;
    int n_wide;              // straddlers 0 .. n_wide - 1 are summed by a whole workgroup each
    int order;               // far-field order: 0 (Alg. 4), 1 or 2 (also writes momhi)
    int scalar;              // the attribute is scalar (set by launch_moments)
    const int2 *gtab;        // MOM_COMB_*: per 64-point group, its parts [x, y) (x = y: whole walk)
    int ngroups;             // MOM_COMB_*: groups
};

struct TravArgs {
    const float4 *tpts;      // targets (sorted), their caller rows and clouds;
    const uint32_t *tperm;   // the points themselves, or sorted query points
    const int32_t *tcloud;
    const float4 *pts;
    const int4 *topo;
    const float4 *mom;
    const float4 *src4;      // sorted vector attributes (A, G)
    const float *srcs;       // sorted scalar attributes (A^T)
    const uint32_t *perm;
    float *out;              // TR_OUT_CALLER: caller-order output
    float *rho;              // TR_RHO output
    float4 *out4;            // TR_R / TR_RESCALE output
    double *partial;         // per-task partial sums (indexed by task_slot)
    unsigned long long *pairs;  // pair counter (counting variant)
    unsigned long long *flips;  // TR_RESCALE: per cloud, updates against mu (or null)
    const float *areas;      // TR_RESCALE: sorted fixed areas (or null: keep |mu|)
    const int32_t *cloud;    // cloud of each sorted point (for flips)
    const int4 *tasks;       // per wavefront: first, last target; first, end node
    const int32_t *task_slot;  // >= 0: group slot (whole walk); < 0: -1 - part slot
    const int32_t *chain;    // per task: ancestors of its first node (kChainStride ints)
    const int32_t *roots;    // first node of each cloud (nclouds + 1)
    float *parts;            // per part slot: 3 x 64 sums rounded to FP32 (component-major)
    int32_t *plan;           // TR_PLAN output, kPlanStride ints per group
    int ntasks;              // wavefronts launched
    int nslots;              // groups: row stride of the per-group partial sums
    int tpl;                 // target groups of 64 per wavefront (1, 2, 4)
    int prefetch;            // software-pipelined node walk
    int n, m;
    const float *momhi;      // far-field moments (order >= 1)
    const float4 *tvec;      // P: each target's own vector (sorted)
    const float *gc;         // TR_POSGRAD: caller-order g
    const float *gradf;      // TR_POSGRAD: caller-order grad F; TR_ACCUM: the base (N,3)
    float w2;
    int order;               // far-field order 0, 1, 2
    double oscale;           // TR_OUT_CALLER: factor on the output (1 unless a caller scales)
    int defer_k;             // defer subtrees needed by at most this many lanes (0: never)
};

}  // namespace wnnc
