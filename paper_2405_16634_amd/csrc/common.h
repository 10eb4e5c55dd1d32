// Internal declarations shared by the library's HIP sources (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/wnnc.h"

namespace wnnc {

constexpr int kWave = 64;
constexpr int kChunk = 256;      // points per moment-pass chunk (one workgroup)
constexpr int kTravBlock = 64;  // traversal workgroup: one wave (finest dispatch)
constexpr int kMaxDepth = 15;    // 15 levels below the root: 45-bit Morton keys

// Node topology, one int4 per node in depth-first pre-order:
//   x = skip: index of the first node after this node's subtree
//   y = begin, z = end: the node's points are sorted positions [begin, end)
//   w = depth | (leaf << 4)
// The first child of an internal node is the next node (index + 1).
__host__ __device__ inline int topo_depth(int meta) { return meta & 15; }
__host__ __device__ inline int topo_leaf(int meta) { return (meta >> 4) & 1; }

// Node record written by every moment pass and read by the traversal, 64
// bytes per node (one 16-dword scalar load):
//   [0] hi(x_B).x, .y, .z, flags (int bits)
//   [1] nu_B (3 floats; a scalar attribute in .x), skip (int bits)
//   [2] lo(x_B).x, .y, .z, (c * width)^2 (the acceptance threshold)
//   [3] first point, end point (int bits), 0, 0
// with x_B = hi + lo to about 2^-48 (hi = FP32 rounding of the FP64 x_B,
// lo = FP32 rounding of the rest), so that target - x_B keeps full FP32
// precision when the target is close to the node.
// flags = depth | leaf << 4 | single-point leaf << 5 | zero weight << 6.
// The traversal addresses records with 32-bit byte offsets: at most
// kMaxNodes nodes.
constexpr int kRecStride = 4;
constexpr int64_t kMaxNodes = int64_t(1) << 26;
constexpr int kRecLeaf = 16;
constexpr int kRecSingle = 32;
constexpr int kRecZero = 64;

enum Op { OP_A = WNNC_OP_A, OP_AT = WNNC_OP_AT, OP_G = WNNC_OP_G };

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
};

// Split planning: the walk of every 64-target group is recorded as its node
// visit count and the node at every kPlanStep-th visit (up to kPlanCap of
// them), kPlanStride ints per group.
constexpr int kPlanStep = 64;
constexpr int kPlanCap = 63;
constexpr int kPlanStride = kPlanCap + 1;

struct MomArgs {
    const float4 *pts;       // sorted points
    const int4 *topo;
    const uint32_t *node_off;
    const int32_t *node_strad;
    const uint32_t *tail_off;
    const int32_t *tail_list;
    const int32_t *strad_node;
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
    double *chunk_tot;       // 8 doubles per chunk
    double *head;            // 8 doubles per straddler
    double *tail;            // 8 doubles per straddler
    float4 *mom;             // node records, kRecStride float4 per node
    float *wout;             // optional: W = sum |nu| per node (inspection)
    float thr2[16];          // (c * 2^(1-d))^2 per depth d, copied into records
    int n;
    int n_strad;
};

struct TravArgs {
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
    const int32_t *cloud;    // cloud of each sorted point (for flips)
    const int4 *tasks;       // per wavefront: first, last target; first, end node
    const int32_t *task_slot;  // >= 0: group slot (whole walk); < 0: -1 - part slot
    const int32_t *roots;    // first node of each cloud (nclouds + 1)
    double *parts;           // per part slot: 3 x 64 FP64 sums (component-major)
    int32_t *plan;           // TR_PLAN output, kPlanStride ints per group
    int ntasks;              // wavefronts launched
    int nslots;              // groups: row stride of the per-group partial sums
    int tpl;                 // target groups of 64 per wavefront (1, 2, 4)
    int prefetch;            // software-pipelined node walk
    int n, m;
    float w2;
    float thr2[16];          // (c * 2^(1-d))^2 per depth d
};

}  // namespace wnnc

// A device array that only grows.
template <typename T>
struct DevBuf {
    T *p = nullptr;
    int64_t cap = 0;
    hipError_t ensure(int64_t need) {
        if (need <= cap && p) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            p = nullptr;
            cap = 0;
            if (e != hipSuccess) return e;
        }
        int64_t c = need + need / 4 + 64;
        hipError_t e = hipMalloc((void **)&p, (size_t)c * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        cap = c;
        return hipSuccess;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

// The context (opaque to callers).
struct wnnc_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    unsigned flags = 0;

    int64_t n = 0, m = 0;
    float c = 2.0f;
    int depth = 15;
    bool built = false;

    // tree (sorted order; nodes in depth-first pre-order)
    DevBuf<float4> pts;            // n sorted normalized points
    DevBuf<uint32_t> perm;         // n: sorted position -> caller index
    DevBuf<int4> topo;             // m
    DevBuf<float4> cells;          // m: node cell box, or the point of a single-point leaf
    DevBuf<uint32_t> node_off;     // n+1: first node started by each point
    DevBuf<int32_t> node_strad;    // m: straddler slot or -1
    DevBuf<int32_t> strad_node;    // n_strad
    int32_t n_strad = 0;
    DevBuf<uint32_t> tail_off;     // chunks+1
    DevBuf<int32_t> tail_list;     // n_strad
    DevBuf<double> chunk_tot;      // 8 per chunk
    DevBuf<double> head, tail;     // 8 per straddler
    DevBuf<float4> mom;            // kRecStride per node
    DevBuf<float> wbuf;            // per-node W, filled on request

    // build scratch
    DevBuf<unsigned long long> keys_a, keys_b;
    DevBuf<uint32_t> vals_b;
    DevBuf<uint32_t> hist;
    DevBuf<uint32_t> scan_tmp;
    DevBuf<uint32_t> u32_tmp;      // n+1
    DevBuf<uint32_t> mflag, mslot; // m+1
    DevBuf<double> norm_tmp;
    DevBuf<int64_t> norm_off;

    // clouds (a single build is one cloud)
    int nclouds = 1;
    std::vector<int64_t> offsets;  // host, nclouds + 1 (caller = sorted ranges)
    std::vector<int32_t> roots;    // host, nclouds + 1: first node of each cloud
    DevBuf<int64_t> d_offsets;     // nclouds + 1
    DevBuf<int32_t> d_roots;       // nclouds + 1
    DevBuf<int32_t> cloud_of;      // n: cloud of each sorted point
    // wavefront tasks for the current tile shape.  A group is 64 * tpl
    // consecutive targets of one cloud; its walk runs as one task, or, split
    // into parts of about `split` node visits, as one task per part plus a
    // combining pass (only for tpl = 1).
    int tpl = 1;
    int prefetch = 0;
    int split = 0;
    int ntasks = 0;                // tasks launched per traversal
    int ngroups = 0;               // groups (per-group partial sums)
    int nparts = 0;                // part slots
    int nsplit = 0;                // groups walked in parts
    DevBuf<int4> tasks;
    DevBuf<int32_t> task_slot;
    DevBuf<int32_t> task_lo;       // nclouds + 1: group range of each cloud
    DevBuf<int4> split_groups;     // nsplit: first, last target; first, end part slot
    DevBuf<int32_t> split_slot;    // nsplit: group slot
    DevBuf<double> parts;          // nparts * 3 * 64
    std::vector<int32_t> plan;     // host: recorded walks of the 64-target groups
    DevBuf<int32_t> d_plan;

    // iteration buffers (sorted order)
    DevBuf<float4> va, vb, vr;
    DevBuf<float> rho;
    DevBuf<double> partial;        // 3 rows of ngroups per-group sums
    DevBuf<double> scalars;        // alpha per cloud
    DevBuf<double> energy;
    int last_energy_count = 0;
    DevBuf<unsigned long long> pair_ctr;  // 3 counters

    // warm start: neighbours, features, MLP activations and scratch
    DevBuf<int4> knn_groups;       // 64-point groups of every cloud (first, last; root, end)
    int knn_ngroups = 0;
    DevBuf<int32_t> knn_idx;       // n * 16 sorted neighbour positions
    DevBuf<float> knn_d2;          // n * 16 squared distances
    DevBuf<float> feat;            // n * 48 features (caller order)
    DevBuf<float> mlp_h1, mlp_h2, mlp_y, mlp_dy, mlp_d1, mlp_d2, mlp_part;
    DevBuf<double> mlp_lpart;
    DevBuf<unsigned long long> flip_ctr;  // per cloud
    DevBuf<float> nhat;            // n * 3 predicted unit normals (caller order)

    // statistics
    int64_t calls[3] = {0, 0, 0};
    double trav_ms[3] = {0, 0, 0};
    double mom_ms = 0;
    double comb_ms = 0;
    double build_ms = 0;

    // event pairs of timed launches, resolved by wnnc_stats
    struct Timed {
        hipEvent_t a, b;
        int kind;  // 0..2 traversal of an operator kind, 3 moment pass, 4 combining pass
    };
    std::vector<Timed> pending;
    std::vector<hipEvent_t> event_pool;
};
