// Internal declarations shared by the library's HIP sources (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/wnnc.h"
#include "layout.h"

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
    int leaf_cap = 1;
    bool built = false;

    // tree (sorted order; nodes in depth-first pre-order)
    DevBuf<float4> pts;            // n sorted normalized points
    DevBuf<uint32_t> perm;         // n: sorted position -> caller index
    DevBuf<int4> topo;             // m
    DevBuf<float4> cells;          // m: node cell box, or the point of a single-point leaf
    DevBuf<uint32_t> node_off;     // n+1: first node started by each point
    DevBuf<int32_t> node_strad;    // m: straddler slot or -1 (build)
    DevBuf<int32_t> strad_node;    // n_strad
    DevBuf<int4> strad_topo;       // n_strad: topology of each straddler
    int32_t n_strad = 0;
    int32_t n_wide = 0;            // straddlers 0 .. n_wide - 1 have more than 64 chunks in between
    DevBuf<uint32_t> tail_off;     // chunks+1
    DevBuf<int2> tail_list;        // n_strad: (straddler slot, end point), by end chunk
    DevBuf<double> chunk_tot;      // kMomSlots per chunk (slot-major)
    DevBuf<double> head, tail;     // kMomSlots per straddler
    DevBuf<float4> mom;            // kRecStride per node
    DevBuf<int2> mnode;            // m: the moment pass's view of each node
    DevBuf<float> wbuf;            // per-node W, filled on request

    // build scratch
    DevBuf<unsigned long long> keys_a, keys_b;
    DevBuf<uint32_t> vals_b;
    DevBuf<uint32_t> hist;
    DevBuf<uint32_t> scan_tmp;
    DevBuf<uint32_t> u32_tmp;      // n+1
    DevBuf<uint32_t> mflag, mslot; // m+1
    DevBuf<uint32_t> wflag, wslot; // m+1
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
    // per operator kind: -1 follows `prefetch`, else the autotuner's choice
    int pf_op[wnnc::kOpKinds] = {-1, -1, -1, -1, -1};
    int split = 256;               // node visits per part of a split walk (0: whole walks)
    int defer_k = 32;              // defer subtrees needed by at most this many lanes (0: never)
    int ntasks = 0;                // tasks launched per traversal
    int ngroups = 0;               // groups (per-group partial sums)
    int nparts = 0;                // part slots
    int nsplit = 0;                // groups walked in parts
    DevBuf<int4> tasks;
    DevBuf<int32_t> task_slot;
    DevBuf<int32_t> task_chain;    // ntasks * kChainStride: ancestors of each task's first node
    DevBuf<int32_t> task_lo;       // nclouds + 1: group range of each cloud
    DevBuf<int4> split_groups;     // nsplit: first, last target; first, end part slot
    DevBuf<int32_t> split_slot;    // nsplit: group slot
    DevBuf<int2> gtab;             // ngroups: part range of each group (when gtab_ok)
    bool gtab_ok = false;          // groups are the 64-point blocks: a moment pass can combine
    DevBuf<float> parts;           // nparts * 3 * 64
    std::vector<int32_t> plan;     // host: recorded walks of the 64-target groups
    DevBuf<int32_t> d_plan;

    // off-surface queries (wnnc_winding_at): sorted copies and their tasks
    DevBuf<unsigned long long> qkeys_a, qkeys_b;
    DevBuf<uint32_t> qperm, qvals_b;
    DevBuf<float4> qpts;
    DevBuf<int4> qtasks;
    DevBuf<int32_t> qslot, qcloud;

    // iteration buffers (sorted order)
    DevBuf<float4> va, vb, vr;
    DevBuf<float> rho;
    DevBuf<float> areas;
    DevBuf<float> momhi;           // far-field moments (far_order >= 1)
    DevBuf<uint32_t> finite_flag;  // WNNC_FLAG_CHECK_FINITE result
    DevBuf<float> gradf;           // caller-order grad F for the position gradient
    int far_order = 0;             // 0: Alg. 4's representative term; 1, 2: Taylor orders
    int far_wsafe = 0;             // accept a node only when its cell is beyond w           // fixed areas (sorted), when an orientation uses them
    DevBuf<double> partial;        // 3 rows of ngroups per-group sums
    DevBuf<double> scalars;        // alpha per cloud
    DevBuf<double> energy;
    int last_energy_count = 0;
    DevBuf<unsigned long long> pair_ctr;  // one counter per operator kind

    // warm start: neighbours, features, MLP activations and scratch
    DevBuf<int4> knn_groups;       // neighbour-search groups (first, last; root, end)
    int knn_ngroups = 0;           // 0: not built for the current tree
    DevBuf<uint32_t> knn_tmp;      // 4 n: group construction
    DevBuf<int32_t> knn_idx;       // n * 16 sorted neighbour positions
    DevBuf<float> knn_d2;          // n * 16 squared distances
    DevBuf<float> feat;            // n * 48 features (caller order)
    DevBuf<float> mlp_h1, mlp_h2, mlp_y, mlp_dy, mlp_d1, mlp_d2, mlp_part;
    DevBuf<double> mlp_lpart;
    DevBuf<unsigned long long> flip_ctr;  // per cloud
    DevBuf<float> nhat;            // n * 3 predicted unit normals (caller order)

    // statistics
    int64_t calls[wnnc::kOpKinds] = {};
    double trav_ms[wnnc::kOpKinds] = {};
    double mom_ms = 0;
    double comb_ms = 0;
    double build_ms = 0;

    // event pairs of timed launches, resolved by wnnc_stats
    struct Timed {
        hipEvent_t a, b;
        // 0..kOpKinds-1 the traversal of an operator kind, then the moment
        // pass and the combining pass
        int kind;
    };
    std::vector<Timed> pending;
    std::vector<hipEvent_t> event_pool;
    // the events of the timed call in progress (null when none is): its
    // first launch carries the start event, its last the stop event
    struct LaunchEvents {
        hipEvent_t start = nullptr, stop = nullptr;
        bool started = false, stopped = false;
    } lev;
};
