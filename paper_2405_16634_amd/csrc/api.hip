// The C ABI (include/wnnc.h): argument checks, buffers, and the order of
// kernel launches for the operators and for the WNNC iteration (Alg. 3).
#include <float.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "common.h"
#include "internal.h"

using namespace wnnc;

namespace {

thread_local std::string g_err;

wnnc_status fail(wnnc_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIPCHK(x)                                                                         \
    do {                                                                                  \
        hipError_t _e = (x);                                                              \
        if (_e != hipSuccess)                                                             \
            return fail(_e == hipErrorOutOfMemory ? WNNC_ENOMEM : WNNC_EDEVICE, "%s: %s", \
                        #x, hipGetErrorString(_e));                                       \
    } while (0)

// The events of one timed call when WNNC_FLAG_TIME_KERNELS is set: the
// call's launches carry them (launch_k), its first launch the start, its
// last the stop.  A call that launched nothing records no time.
struct Timed {
    wnnc_ctx_s *ctx;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(wnnc_ctx_s *c, int k) : ctx(c), kind(k) {
        const bool on = (ctx->flags & WNNC_FLAG_TIME_KERNELS) ||
                        ((ctx->flags & WNNC_FLAG_TIME_TRAVERSAL) && kind < kOpKinds);
        if (!on) return;
        a = get();
        b = get();
        if (a && b) {
            ctx->lev = wnnc_ctx_s::LaunchEvents();
            ctx->lev.start = a;
            ctx->lev.stop = b;
        }
    }
    hipEvent_t get() {
        if (!ctx->event_pool.empty()) {
            hipEvent_t e = ctx->event_pool.back();
            ctx->event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void done() {
        const bool recorded = ctx->lev.started && ctx->lev.stopped;
        ctx->lev = wnnc_ctx_s::LaunchEvents();
        if (recorded) {
            ctx->pending.push_back({a, b, kind});
        } else {
            if (a) ctx->event_pool.push_back(a);
            if (b) ctx->event_pool.push_back(b);
        }
        a = b = nullptr;
    }
    // an early return (a failed launch) still closes the call
    ~Timed() {
        if (a || b) done();
    }
};

// Squared acceptance distance per depth: (c 2^(1-d))^2 (Alg. 4), or with
// the cutoff-safe test also at least (w + sqrt(3) 2^(1-d))^2, so that an
// accepted node's cell holds no point closer to the target than w.
static void fill_thresholds(const wnnc_ctx_s *c, float w, bool wsafe, float *thr2) {
    for (int d = 0; d < 16; ++d) {
        const double width = ldexp(2.0, -d);
        double t = (double)c->c * width;
        if (wsafe) t = fmax(t, (double)w + sqrt(3.0) * width);
        thr2[d] = (float)(t * t);
    }
}

// Moment-pass arguments for an operator call at width w (paper = true:
// Alg. 4's far field whatever the context's far-field setting).
MomArgs mom_args(wnnc_ctx_s *c, float w, bool paper = false) {
    // (fields not set here are per-call inputs and outputs)
    MomArgs a;
    memset(&a, 0, sizeof(a));
    a.pts = c->pts.p;
    a.mnode = c->mnode.p;
    a.node_off = c->node_off.p;
    a.tail_off = c->tail_off.p;
    a.tail_list = c->tail_list.p;
    a.strad_node = c->strad_node.p;
    a.strad_topo = c->strad_topo.p;
    a.perm = c->perm.p;
    a.chunk_tot = c->chunk_tot.p;
    a.head = c->head.p;
    a.tail = c->tail.p;
    a.mom = c->mom.p;
    a.cloud = c->cloud_of.p;
    a.alpha = c->scalars.p;
    a.n = (int)c->n;
    a.n_strad = c->n_strad;
    a.n_wide = c->n_wide;
    fill_thresholds(c, w, c->far_wsafe && !paper, a.thr2);
    a.order = paper ? 0 : c->far_order;
    a.momhi = a.order > 0 ? c->momhi.p : nullptr;
    return a;
}

TravArgs trav_args(wnnc_ctx_s *c, float w) {
    TravArgs a;
    memset(&a, 0, sizeof(a));
    a.tpts = c->pts.p;
    a.tperm = c->perm.p;
    a.tcloud = c->cloud_of.p;
    a.pts = c->pts.p;
    a.topo = c->topo.p;
    a.mom = c->mom.p;
    a.perm = c->perm.p;
    a.pairs = c->pair_ctr.p;
    a.cloud = c->cloud_of.p;
    a.tasks = c->tasks.p;
    a.task_slot = c->task_slot.p;
    a.chain = c->task_chain.p;
    a.roots = c->d_roots.p;
    a.parts = c->parts.p;
    a.ntasks = c->ntasks;
    a.nslots = c->ngroups;
    a.tpl = c->tpl;
    a.prefetch = c->prefetch;
    a.n = (int)c->n;
    a.m = (int)c->m;
    // pairs closer than w, and coincident pairs, contribute nothing
    a.w2 = fmaxf((float)((double)w * (double)w), FLT_MIN);
    a.order = c->far_order;
    a.momhi = c->far_order > 0 ? c->momhi.p : nullptr;
    a.oscale = 1.0;
    a.defer_k = c->defer_k;
    return a;
}

// The traversal addresses a node's far-field moments (kHiStride floats) with
// a 32-bit byte offset.
constexpr int64_t kMaxHiNodes = (int64_t(1) << 32) / (kHiStride * 4);

// Timed kinds: 0..kOpKinds-1 the traversal of each operator, then these two.
constexpr int kKindMoments = kOpKinds, kKindCombine = kOpKinds + 1;

wnnc_status run_moments(wnnc_ctx_s *c, MomMode mode, const MomArgs &a) {
    Timed tm(c, kKindMoments);
    HIPCHK(launch_moments(c, mode, a));
    tm.done();
    return WNNC_OK;
}

// The walk an operator kind uses: the prefetching one or the plain one.
int prefetch_of(const wnnc_ctx_s *c, Op op) { return c->pf_op[op] >= 0 ? c->pf_op[op] : c->prefetch; }

// The walk and its combining pass; without the combining pass (combine =
// false) the moment pass that follows runs it (run_moments_comb with the
// same arguments).
wnnc_status run_traverse(wnnc_ctx_s *c, Op op, TravMode mode, const TravArgs &args,
                         bool combine = true) {
    TravArgs a = args;
    a.prefetch = prefetch_of(c, op);
    Timed tm(c, (int)op);
    HIPCHK(launch_traverse(c, op, mode, (c->flags & WNNC_FLAG_COUNT_PAIRS) != 0, a));
    tm.done();
    if (combine) {
        Timed tc(c, kKindCombine);
        HIPCHK(launch_combine(c, op, mode, a));
        tc.done();
    }
    c->calls[op] += 1;
    return WNNC_OK;
}

wnnc_status run_moments_comb(wnnc_ctx_s *c, MomMode mode, const MomArgs &ma, Op op,
                             const TravArgs &walk) {
    MomArgs a = ma;
    a.gtab = c->gtab.p;
    a.ngroups = c->ngroups;
    TravArgs t = walk;
    t.prefetch = prefetch_of(c, op);
    Timed tm(c, kKindMoments);
    HIPCHK(launch_moments_comb(c, mode, a, t));
    tm.done();
    return WNNC_OK;
}

bool finite_nonneg(float w) { return isfinite(w) && w >= 0.0f; }

#define CHECK_CTX(ctx)                                                          \
    do {                                                                        \
        if (!(ctx)) return fail(WNNC_EINVAL, "null context");                   \
        HIPCHK(hipSetDevice((ctx)->device));                                    \
    } while (0)

#define CHECK_BUILT(ctx)                                                                  \
    do {                                                                                  \
        if (!(ctx)->built) return fail(WNNC_ESTATE, "no tree: call wnnc_build first");    \
    } while (0)

#define RETURN_IF(x)                  \
    do {                              \
        wnnc_status _s = (x);         \
        if (_s != WNNC_OK) return _s; \
    } while (0)

}  // namespace

extern "C" {

const char *wnnc_last_error(void) { return g_err.c_str(); }

const char *wnnc_version(void) { return "wnnc-mi355x 0.1 (gfx950)"; }

wnnc_status wnnc_create(wnnc_ctx *out, int device, void *stream) {
    if (!out) return fail(WNNC_EINVAL, "out is null");
    *out = nullptr;
    int count = 0;
    HIPCHK(hipGetDeviceCount(&count));
    if (device < 0 || device >= count)
        return fail(WNNC_EINVAL, "device %d out of range (%d devices)", device, count);
    {
        // the no-allocation entry points' scratch: its device address, once
        // per device, with that device current
        int prev = 0;
        HIPCHK(hipGetDevice(&prev));
        HIPCHK(hipSetDevice(device));
        const hipError_t e = noalloc_setup(device);
        HIPCHK(hipSetDevice(prev));
        HIPCHK(e);
    }
    wnnc_ctx_s *c = new (std::nothrow) wnnc_ctx_s();
    if (!c) return fail(WNNC_ENOMEM, "host allocation failed");
    c->device = device;
    c->stream = (hipStream_t)stream;
    *out = c;
    return WNNC_OK;
}

wnnc_status wnnc_destroy(wnnc_ctx ctx) {
    if (!ctx) return WNNC_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->pts.release();
    ctx->perm.release();
    ctx->topo.release();
    ctx->node_off.release();
    ctx->node_strad.release();
    ctx->strad_node.release();
    ctx->strad_topo.release();
    ctx->gtab.release();
    ctx->wflag.release();
    ctx->wslot.release();
    ctx->tail_off.release();
    ctx->tail_list.release();
    ctx->chunk_tot.release();
    ctx->head.release();
    ctx->tail.release();
    ctx->mom.release();
    ctx->mnode.release();
    ctx->keys_a.release();
    ctx->keys_b.release();
    ctx->vals_b.release();
    ctx->hist.release();
    ctx->scan_tmp.release();
    ctx->u32_tmp.release();
    ctx->mflag.release();
    ctx->mslot.release();
    ctx->norm_tmp.release();
    ctx->va.release();
    ctx->vb.release();
    ctx->vr.release();
    ctx->rho.release();
    ctx->partial.release();
    ctx->scalars.release();
    ctx->energy.release();
    ctx->pair_ctr.release();
    ctx->wbuf.release();
    ctx->d_offsets.release();
    ctx->d_roots.release();
    ctx->norm_off.release();
    ctx->cloud_of.release();
    ctx->tasks.release();
    ctx->task_slot.release();
    ctx->task_chain.release();
    ctx->task_lo.release();
    ctx->knn_groups.release();
    ctx->knn_tmp.release();
    ctx->areas.release();
    ctx->momhi.release();
    ctx->gradf.release();
    ctx->qkeys_a.release();
    ctx->qkeys_b.release();
    ctx->qperm.release();
    ctx->qvals_b.release();
    ctx->qpts.release();
    ctx->qtasks.release();
    ctx->qslot.release();
    ctx->qcloud.release();
    ctx->cells.release();
    ctx->knn_idx.release();
    ctx->knn_d2.release();
    ctx->feat.release();
    ctx->mlp_h1.release();
    ctx->mlp_h2.release();
    ctx->mlp_y.release();
    ctx->mlp_dy.release();
    ctx->mlp_d1.release();
    ctx->mlp_d2.release();
    ctx->mlp_part.release();
    ctx->mlp_lpart.release();
    ctx->flip_ctr.release();
    ctx->nhat.release();
    for (auto &t : ctx->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    delete ctx;
    return WNNC_OK;
}

wnnc_status wnnc_set_stream(wnnc_ctx ctx, void *stream) {
    CHECK_CTX(ctx);
    ctx->stream = (hipStream_t)stream;
    return WNNC_OK;
}

wnnc_status wnnc_set_flags(wnnc_ctx ctx, unsigned flags) {
    CHECK_CTX(ctx);
    if (flags & ~(WNNC_FLAG_COUNT_PAIRS | WNNC_FLAG_TIME_KERNELS | WNNC_FLAG_CHECK_FINITE |
                  WNNC_FLAG_TIME_TRAVERSAL | WNNC_FLAG_SEPARATE_COMBINE))
        return fail(WNNC_EINVAL, "unknown flags 0x%x", flags);
    ctx->flags = flags;
    return WNNC_OK;
}

// With WNNC_FLAG_CHECK_FINITE: WNNC_ENUMERIC if any of the n floats at p
// (device) is NaN or infinite (synchronizes); WNNC_OK otherwise, and always
// without the flag or for a null p.
static wnnc_status check_finite(wnnc_ctx_s *ctx, const float *p, int64_t n, const char *name) {
    if (!(ctx->flags & WNNC_FLAG_CHECK_FINITE) || !p || n <= 0) return WNNC_OK;
    HIPCHK(ctx->finite_flag.ensure(1));
    HIPCHK(hipMemsetAsync(ctx->finite_flag.p, 0, sizeof(uint32_t), ctx->stream));
    HIPCHK(launch_check_finite(p, n, ctx->finite_flag.p, ctx->stream));
    uint32_t bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, ctx->finite_flag.p, sizeof(bad), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (bad) return fail(WNNC_ENUMERIC, "%s holds a NaN or an infinity", name);
    return WNNC_OK;
}

static wnnc_status check_offsets(const int64_t *offsets, int B, int64_t *N) {
    if (!offsets) return fail(WNNC_EINVAL, "null offsets");
    if (B < 1 || B > (1 << 18)) return fail(WNNC_EINVAL, "cloud count %d out of range 1..2^18", B);
    if (offsets[0] != 0) return fail(WNNC_EINVAL, "offsets[0] must be 0");
    for (int c = 0; c < B; ++c)
        if (offsets[c + 1] <= offsets[c]) return fail(WNNC_EINVAL, "cloud %d is empty", c);
    *N = offsets[B];
    if (*N > INT32_MAX - 1) return fail(WNNC_EINVAL, "N = %lld out of range", (long long)*N);
    return WNNC_OK;
}

static wnnc_status normalize_impl(wnnc_ctx ctx, const float *P, const int64_t *offsets, int B,
                                  float *P_norm, double *center_scale) {
    int64_t N = 0;
    RETURN_IF(check_offsets(offsets, B, &N));
    if (!P || !P_norm) return fail(WNNC_EINVAL, "null point pointer");
    RETURN_IF(check_finite(ctx, P, 3 * N, "P"));
    HIPCHK(ctx->norm_tmp.ensure(normalize_tmp_doubles(B)));
    HIPCHK(ctx->norm_off.ensure(B + 1));
    HIPCHK(hipMemcpyAsync(ctx->norm_off.p, offsets, (size_t)(B + 1) * sizeof(int64_t),
                          hipMemcpyHostToDevice, ctx->stream));
    const int64_t at = launch_normalize(P, N, ctx->norm_off.p, B, P_norm, ctx->norm_tmp.p, ctx->stream);
    HIPCHK(hipGetLastError());
    std::vector<double> cs((size_t)4 * B);
    HIPCHK(hipMemcpyAsync(cs.data(), ctx->norm_tmp.p + at, cs.size() * sizeof(double),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (center_scale) memcpy(center_scale, cs.data(), cs.size() * sizeof(double));
    return WNNC_OK;
}

wnnc_status wnnc_normalize(wnnc_ctx ctx, const float *P, int64_t N, float *P_norm,
                           double *center_scale) {
    CHECK_CTX(ctx);
    if (N < 1 || N > INT32_MAX - 1) return fail(WNNC_EINVAL, "N = %lld out of range", (long long)N);
    const int64_t off[2] = {0, N};
    return normalize_impl(ctx, P, off, 1, P_norm, center_scale);
}

wnnc_status wnnc_normalize_batched(wnnc_ctx ctx, const float *P, const int64_t *offsets, int B,
                                   float *P_norm, double *center_scale) {
    CHECK_CTX(ctx);
    return normalize_impl(ctx, P, offsets, B, P_norm, center_scale);
}

// Records the walk of every 64-target group (node visits of the adjoint
// traversal with the constant attribute 1/2: every weight is positive, so
// it visits the nodes a smooth attribute would) for splitting long walks.
static hipError_t plan_walks(wnnc_ctx_s *ctx) {
    ctx->plan.clear();
    TRY(make_tasks(ctx, 1, 0));
    ctx->knn_ngroups = 0;  // the neighbour search builds its groups on first use
    const int64_t len = (int64_t)ctx->ngroups * kPlanStride;
    TRY(ctx->d_plan.ensure(len));
    TRY(hipMemsetAsync(ctx->d_plan.p, 0, (size_t)len * sizeof(int32_t), ctx->stream));
    MomArgs ma = mom_args(ctx, 0.0f);
    ma.order = 0;  // the walk plan follows Alg. 4's acceptance only
    ma.outs = ctx->rho.p;
    TRY(launch_moments(ctx, MOM_CONST_HALF, ma));
    TravArgs ta = trav_args(ctx, 0.0f);
    ta.order = 0;
    ta.srcs = ctx->rho.p;
    ta.plan = ctx->d_plan.p;
    TRY(record_plan(ctx, ta));
    std::vector<int32_t> pl((size_t)len);
    TRY(hipMemcpyAsync(pl.data(), ctx->d_plan.p, (size_t)len * sizeof(int32_t),
                       hipMemcpyDeviceToHost, ctx->stream));
    TRY(hipStreamSynchronize(ctx->stream));
    ctx->plan.swap(pl);
    return hipSuccess;
}

static wnnc_status build_impl(wnnc_ctx ctx, const float *P, const int64_t *offsets, int B,
                              const wnnc_tree_opts *opts) {
    int64_t N = 0;
    RETURN_IF(check_offsets(offsets, B, &N));
    if (!P) return fail(WNNC_EINVAL, "null point pointer");
    wnnc_tree_opts o = {2.0f, 15, 1};
    if (opts) o = *opts;
    if (!(isfinite(o.c) && o.c > 0.0f)) return fail(WNNC_EINVAL, "c must be finite and > 0");
    if (o.max_depth < 1 || o.max_depth > kMaxDepth)
        return fail(WNNC_EINVAL, "max_depth must be in 1..15");
    if (o.leaf_cap < 1 || o.leaf_cap > 256) return fail(WNNC_EINVAL, "leaf_cap must be in 1..256");
    RETURN_IF(check_finite(ctx, P, 3 * N, "P"));
    ctx->built = false;
    ctx->n = N;
    ctx->c = o.c;
    ctx->depth = o.max_depth;
    ctx->leaf_cap = o.leaf_cap;
    ctx->nclouds = B;
    ctx->offsets.assign(offsets, offsets + B + 1);
    HIPCHK(ctx->d_offsets.ensure(B + 1));
    HIPCHK(hipMemcpyAsync(ctx->d_offsets.p, ctx->offsets.data(), (size_t)(B + 1) * sizeof(int64_t),
                          hipMemcpyHostToDevice, ctx->stream));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, ctx->stream));
    const int tpl = ctx->tpl, split = ctx->split;  // planning uses its own tasks
    hipError_t e = build_tree(ctx, P);
    if (e == hipSuccess) e = plan_walks(ctx);
    if (e == hipSuccess) e = make_tasks(ctx, tpl, split);
    const bool hi_too_big = e == hipSuccess && ctx->far_order > 0 && ctx->m > kMaxHiNodes;
    if (e == hipSuccess && ctx->far_order > 0 && !hi_too_big)
        e = ctx->momhi.ensure(ctx->m * kHiStride);
    if (hi_too_big) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        ctx->built = false;
        return fail(WNNC_EINVAL, "tree build: %lld nodes; the far field of order > 0 takes at most %lld",
                    (long long)ctx->m, (long long)kMaxHiNodes);
    }
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (e == hipErrorNotSupported)
            return fail(WNNC_EINVAL, "tree build: more than %lld nodes", (long long)kMaxNodes);
        return fail(e == hipErrorOutOfMemory ? WNNC_ENOMEM : WNNC_EDEVICE, "tree build: %s",
                    hipGetErrorString(e));
    }
    HIPCHK(hipEventRecord(e1, ctx->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->build_ms = ms;
    ctx->built = true;
    return WNNC_OK;
}

wnnc_status wnnc_build(wnnc_ctx ctx, const float *P, int64_t N, const wnnc_tree_opts *opts) {
    CHECK_CTX(ctx);
    if (N < 1 || N > INT32_MAX - 1) return fail(WNNC_EINVAL, "N = %lld out of range", (long long)N);
    const int64_t off[2] = {0, N};
    return build_impl(ctx, P, off, 1, opts);
}

wnnc_status wnnc_build_batched(wnnc_ctx ctx, const float *P, const int64_t *offsets, int B,
                               const wnnc_tree_opts *opts) {
    CHECK_CTX(ctx);
    return build_impl(ctx, P, offsets, B, opts);
}

wnnc_status wnnc_set_tile(wnnc_ctx ctx, int tpl) {
    CHECK_CTX(ctx);
    if (tpl != 1 && tpl != 2 && tpl != 4) return fail(WNNC_EINVAL, "tile must be 1, 2 or 4");
    if (ctx->built) {
        hipError_t e = make_tasks(ctx, tpl, ctx->split);
        if (e != hipSuccess) return fail(WNNC_EDEVICE, "tasks: %s", hipGetErrorString(e));
    } else {
        ctx->tpl = tpl;
    }
    return WNNC_OK;
}

wnnc_status wnnc_set_split(wnnc_ctx ctx, int visits) {
    CHECK_CTX(ctx);
    if (visits < 0 || visits > WNNC_MAX_SPLIT)
        return fail(WNNC_EINVAL, "split must be in 0..%d", WNNC_MAX_SPLIT);
    if (ctx->built) {
        hipError_t e = make_tasks(ctx, ctx->tpl, visits);
        if (e != hipSuccess) return fail(WNNC_EDEVICE, "tasks: %s", hipGetErrorString(e));
    } else {
        ctx->split = visits;
    }
    return WNNC_OK;
}

wnnc_status wnnc_set_far_field(wnnc_ctx ctx, int order, int wsafe) {
    CHECK_CTX(ctx);
    if (order < 0 || order > 2) return fail(WNNC_EINVAL, "far-field order must be 0, 1 or 2");
    if (wsafe != 0 && wsafe != 1) return fail(WNNC_EINVAL, "wsafe must be 0 or 1");
    if (order > 0 && ctx->built && ctx->m > kMaxHiNodes)
        return fail(WNNC_EINVAL, "the far field of order > 0 takes at most %lld nodes (tree: %lld)",
                    (long long)kMaxHiNodes, (long long)ctx->m);
    if (order > 0 && ctx->built) HIPCHK(ctx->momhi.ensure(ctx->m * kHiStride));
    ctx->far_order = order;
    ctx->far_wsafe = wsafe;
    return WNNC_OK;
}

wnnc_status wnnc_get_far_field(wnnc_ctx ctx, int *order, int *wsafe) {
    CHECK_CTX(ctx);
    if (!order || !wsafe) return fail(WNNC_EINVAL, "null output");
    *order = ctx->far_order;
    *wsafe = ctx->far_wsafe;
    return WNNC_OK;
}

wnnc_status wnnc_get_split(wnnc_ctx ctx, int *visits) {
    CHECK_CTX(ctx);
    if (!visits) return fail(WNNC_EINVAL, "null output");
    *visits = ctx->split;
    return WNNC_OK;
}

wnnc_status wnnc_get_tile(wnnc_ctx ctx, int *tpl) {
    CHECK_CTX(ctx);
    if (!tpl) return fail(WNNC_EINVAL, "null output");
    *tpl = ctx->tpl;
    return WNNC_OK;
}

wnnc_status wnnc_set_defer(wnnc_ctx ctx, int lanes) {
    CHECK_CTX(ctx);
    if (lanes < 0 || lanes > kWave) return fail(WNNC_EINVAL, "lanes must be in 0..64");
    ctx->defer_k = lanes;
    return WNNC_OK;
}

wnnc_status wnnc_get_defer(wnnc_ctx ctx, int *lanes) {
    CHECK_CTX(ctx);
    if (!lanes) return fail(WNNC_EINVAL, "null lanes");
    *lanes = ctx->defer_k;
    return WNNC_OK;
}

wnnc_status wnnc_set_prefetch(wnnc_ctx ctx, int on) {
    CHECK_CTX(ctx);
    ctx->prefetch = on ? 1 : 0;
    for (int k = 0; k < kOpKinds; ++k) ctx->pf_op[k] = -1;
    return WNNC_OK;
}

static wnnc_status run_iterations(wnnc_ctx ctx, int iters, float w1, float w2, int start, int stop,
                                  bool zero, unsigned long long *flips, int sched,
                                  const float *areas);

wnnc_status wnnc_autotune(wnnc_ctx ctx, float w, wnnc_tile_time *times_out) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    if (!finite_nonneg(w)) return fail(WNNC_EINVAL, "w must be finite and >= 0");
    for (int k = 0; k < kOpKinds; ++k) ctx->pf_op[k] = -1;
    // (tpl, split) pairs, each with and without prefetch
    static const int cand[WNNC_AUTOTUNE_CONFIGS / 2][2] = {
        {1, 0}, {2, 0}, {4, 0}, {1, 1024}, {1, 512}, {1, 256}, {1, 128}, {1, 64}};
    double best_ms = 1e300;
    int best = ctx->tpl, best_pf = ctx->prefetch, best_split = ctx->split;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // Each setting times what it is for: kTuneIters iterations of Alg. 3 at
    // width w from mu = 0 (moment passes, A, A^T, A and G in their real mix
    // and on the records the iteration makes).  The first run warms the
    // caches; then the fastest of kTuneReps.
    constexpr int kTuneIters = 3, kTuneReps = 2;
    // the time per iteration of the tasks in place with prefetch pf: the
    // fastest of reps runs after a warm-up
    auto time_setting = [&](int pf, int reps, double *t) -> wnnc_status {
        ctx->prefetch = pf;
        *t = 1e300;
        for (int rep = 0; rep <= reps; ++rep) {
            HIPCHK(launch_zero_f4(ctx->va.p, ctx->n, ctx->stream));
            HIPCHK(hipEventRecord(e0, ctx->stream));
            RETURN_IF(run_iterations(ctx, kTuneIters, w, w, 1, kTuneIters, true, nullptr,
                                     WNNC_SCHEDULE_LINEAR, nullptr));
            HIPCHK(hipEventRecord(e1, ctx->stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) *t = std::min(*t, (double)ms / kTuneIters);
        }
        return WNNC_OK;
    };
    double tk[WNNC_AUTOTUNE_CONFIGS];
    for (int k = 0; k < WNNC_AUTOTUNE_CONFIGS / 2; ++k) {
        hipError_t e = make_tasks(ctx, cand[k][0], cand[k][1]);
        if (e != hipSuccess) return fail(WNNC_EDEVICE, "tasks: %s", hipGetErrorString(e));
        for (int pf = 0; pf < 2; ++pf) {
            double t;
            RETURN_IF(time_setting(pf, kTuneReps, &t));
            tk[2 * k + pf] = t;
            if (times_out) {
                wnnc_tile_time &o = times_out[2 * k + pf];
                o.tpl = cand[k][0];
                o.prefetch = pf;
                o.split = cand[k][1];
                o.ms = t;
            }
        }
    }
    // Settings within 3 % of the fastest are timed again, in turn over
    // kRetimeRounds rounds (so that a drift of the clock between the first
    // timings cannot decide), each keeping its fastest run; then, in list
    // order, a later setting must be faster by more than 1 %: the choice
    // stays put between settings within run-to-run noise.
    constexpr int kRetimeRounds = 3;
    {
        double t0 = 1e300;
        for (int c = 0; c < WNNC_AUTOTUNE_CONFIGS; ++c) t0 = std::min(t0, tk[c]);
        std::vector<int> near;
        for (int c = 0; c < WNNC_AUTOTUNE_CONFIGS; ++c)
            if (tk[c] <= 1.03 * t0) near.push_back(c);
        if (near.size() > 1) {
            for (int round = 0; round < kRetimeRounds; ++round) {
                for (int c : near) {
                    hipError_t e = make_tasks(ctx, cand[c / 2][0], cand[c / 2][1]);
                    if (e != hipSuccess) return fail(WNNC_EDEVICE, "tasks: %s", hipGetErrorString(e));
                    double t;
                    RETURN_IF(time_setting(c % 2, 1, &t));
                    tk[c] = std::min(tk[c], t);
                }
            }
        }
        if (times_out)
            for (int c = 0; c < WNNC_AUTOTUNE_CONFIGS; ++c) times_out[c].ms = tk[c];
        for (int c = 0; c < WNNC_AUTOTUNE_CONFIGS; ++c) {
            if (tk[c] < best_ms * 0.99) {
                best_ms = tk[c];
                best = cand[c / 2][0];
                best_pf = c % 2;
                best_split = cand[c / 2][1];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->prefetch = best_pf;
    hipError_t e = make_tasks(ctx, best, best_split);
    if (e != hipSuccess) return fail(WNNC_EDEVICE, "tasks: %s", hipGetErrorString(e));
    // Then the walk per operator on the chosen tiles: the same iterations
    // with each operator's traversal launches timed (the events ride on the
    // launches), without and with prefetch; an operator takes the other
    // walk than the chosen one only if that is faster by more than 1 %.  The
    // caller's instrumentation is put back afterwards.
    double t_op[2][kOpKinds] = {};
    {
        const unsigned saved_flags = ctx->flags;
        std::vector<wnnc_ctx_s::Timed> saved_pending;
        saved_pending.swap(ctx->pending);
        double saved_ms[kOpKinds];
        int64_t saved_calls[kOpKinds];
        for (int k = 0; k < kOpKinds; ++k) saved_ms[k] = ctx->trav_ms[k], saved_calls[k] = ctx->calls[k];
        wnnc_status st = WNNC_OK;
        for (int pf = 0; pf < 2 && st == WNNC_OK; ++pf) {
            ctx->prefetch = pf;
            for (int k = 0; k < kOpKinds; ++k) t_op[pf][k] = 1e300;
            for (int rep = 0; rep <= kTuneReps && st == WNNC_OK; ++rep) {
                ctx->flags = rep > 0 ? WNNC_FLAG_TIME_TRAVERSAL : 0u;
                hipError_t he = launch_zero_f4(ctx->va.p, ctx->n, ctx->stream);
                if (he == hipSuccess) {
                    st = run_iterations(ctx, kTuneIters, w, w, 1, kTuneIters, true, nullptr,
                                        WNNC_SCHEDULE_LINEAR, nullptr);
                    he = hipStreamSynchronize(ctx->stream);
                }
                if (he != hipSuccess && st == WNNC_OK)
                    st = fail(WNNC_EDEVICE, "autotune: %s", hipGetErrorString(he));
                double sum[kOpKinds] = {};
                for (auto &t : ctx->pending) {
                    float ms = 0.f;
                    if (st == WNNC_OK && t.kind < kOpKinds &&
                        hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess)
                        sum[t.kind] += ms;
                    ctx->event_pool.push_back(t.a);
                    ctx->event_pool.push_back(t.b);
                }
                ctx->pending.clear();
                if (rep > 0)
                    for (int k = 0; k < kOpKinds; ++k) t_op[pf][k] = std::min(t_op[pf][k], sum[k]);
            }
        }
        ctx->flags = saved_flags;
        ctx->pending.swap(saved_pending);
        for (int k = 0; k < kOpKinds; ++k) ctx->trav_ms[k] = saved_ms[k], ctx->calls[k] = saved_calls[k];
        ctx->prefetch = best_pf;
        if (st != WNNC_OK) return st;
    }
    for (int k = 0; k < kOpKinds; ++k) {
        const int other = 1 - best_pf;
        if (t_op[other][k] > 0.0 && t_op[other][k] < 0.99 * t_op[best_pf][k]) ctx->pf_op[k] = other;
    }
    return WNNC_OK;
}

wnnc_status wnnc_winding(wnnc_ctx ctx, const float *n, const float *sigma, float w, float *s_out) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    if (!n || !s_out) return fail(WNNC_EINVAL, "null pointer");
    if (!finite_nonneg(w)) return fail(WNNC_EINVAL, "w must be finite and >= 0");
    RETURN_IF(check_finite(ctx, n, 3 * ctx->n, "n"));
    RETURN_IF(check_finite(ctx, sigma, ctx->n, "sigma"));
    MomArgs ma = mom_args(ctx, w);
    ma.cn = n;
    ma.csig = sigma;
    ma.out4 = ctx->va.p;
    RETURN_IF(run_moments(ctx, MOM_VEC_CALLER, ma));
    TravArgs ta = trav_args(ctx, w);
    ta.src4 = ctx->va.p;
    ta.out = s_out;
    return run_traverse(ctx, OP_A, TR_OUT_CALLER, ta);
}

wnnc_status wnnc_winding_at(wnnc_ctx ctx, const float *n, const float *sigma, float w,
                            const float *Q, int64_t M, float *s_out) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    if (!n || !Q || !s_out) return fail(WNNC_EINVAL, "null pointer");
    if (M < 1 || M > INT32_MAX - 1) return fail(WNNC_EINVAL, "M = %lld out of range", (long long)M);
    if (!finite_nonneg(w)) return fail(WNNC_EINVAL, "w must be finite and >= 0");
    if (ctx->nclouds != 1) return fail(WNNC_EINVAL, "queries need a tree of one cloud");
    RETURN_IF(check_finite(ctx, n, 3 * ctx->n, "n"));
    RETURN_IF(check_finite(ctx, sigma, ctx->n, "sigma"));
    RETURN_IF(check_finite(ctx, Q, 3 * M, "Q"));
    hipStream_t st = ctx->stream;
    MomArgs ma = mom_args(ctx, w);
    ma.cn = n;
    ma.csig = sigma;
    ma.out4 = ctx->va.p;
    RETURN_IF(run_moments(ctx, MOM_VEC_CALLER, ma));
    // queries in Morton order, 64 per wavefront, whole walks of the tree
    HIPCHK(sort_queries(ctx, Q, M));
    const int ng = (int)((M + kWave - 1) / kWave);
    std::vector<int4> tk((size_t)ng);
    std::vector<int32_t> slot((size_t)ng);
    for (int g = 0; g < ng; ++g) {
        const int64_t f = (int64_t)g * kWave;
        tk[g] = make_int4((int)f, (int)(f + kWave < M ? f + kWave : M), ctx->roots[0], ctx->roots[1]);
        slot[g] = g;
    }
    HIPCHK(ctx->qtasks.ensure(ng));
    HIPCHK(ctx->qslot.ensure(ng));
    HIPCHK(ctx->qcloud.ensure(M));
    HIPCHK(hipMemcpyAsync(ctx->qtasks.p, tk.data(), (size_t)ng * sizeof(int4), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ctx->qslot.p, slot.data(), (size_t)ng * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(ctx->qcloud.p, 0, (size_t)M * sizeof(int32_t), st));
    TravArgs ta = trav_args(ctx, w);
    ta.src4 = ctx->va.p;
    ta.out = s_out;
    ta.tpts = ctx->qpts.p;
    ta.tperm = ctx->qperm.p;
    ta.tcloud = ctx->qcloud.p;
    ta.tasks = ctx->qtasks.p;
    ta.task_slot = ctx->qslot.p;
    ta.ntasks = ng;
    ta.nslots = ng;
    ta.tpl = 1;
    {
        ta.prefetch = prefetch_of(ctx, OP_A);
        Timed tm(ctx, (int)OP_A);
        HIPCHK(launch_traverse(ctx, OP_A, TR_OUT_CALLER, (ctx->flags & WNNC_FLAG_COUNT_PAIRS) != 0, ta));
        tm.done();
        ctx->calls[OP_A] += 1;
    }
    // the host task list is released on return
    HIPCHK(hipStreamSynchronize(st));
    return WNNC_OK;
}

wnnc_status wnnc_gradient(wnnc_ctx ctx, const float *n, const float *sigma, float w,
                          float *grad_out) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    if (!n || !grad_out) return fail(WNNC_EINVAL, "null pointer");
    if (!finite_nonneg(w)) return fail(WNNC_EINVAL, "w must be finite and >= 0");
    RETURN_IF(check_finite(ctx, n, 3 * ctx->n, "n"));
    RETURN_IF(check_finite(ctx, sigma, ctx->n, "sigma"));
    MomArgs ma = mom_args(ctx, w);
    ma.cn = n;
    ma.csig = sigma;
    ma.out4 = ctx->va.p;
    RETURN_IF(run_moments(ctx, MOM_VEC_CALLER, ma));
    TravArgs ta = trav_args(ctx, w);
    ta.src4 = ctx->va.p;
    ta.out = grad_out;
    return run_traverse(ctx, OP_G, TR_OUT_CALLER, ta);
}

}  // extern "C"

// The position gradient of sum_i g_i A(mu)_i (wnnc_winding_grad_x) with the
// caller-order grad F kept in `gradf` (3 N floats of scratch); allocates
// nothing after a build.
static wnnc_status winding_grad_x_impl(wnnc_ctx ctx, const float *n, const float *sigma, float w,
                                       const float *g, float *dx_out, float *gradf) {
    if (!n || !g || !dx_out) return fail(WNNC_EINVAL, "null pointer");
    if (!finite_nonneg(w)) return fail(WNNC_EINVAL, "w must be finite and >= 0");
    RETURN_IF(check_finite(ctx, n, 3 * ctx->n, "n"));
    RETURN_IF(check_finite(ctx, sigma, ctx->n, "sigma"));
    RETURN_IF(check_finite(ctx, g, ctx->n, "g"));
    // grad F(x_k; mu), caller order
    MomArgs ma = mom_args(ctx, w, true);
    ma.cn = n;
    ma.csig = sigma;
    ma.out4 = ctx->va.p;
    RETURN_IF(run_moments(ctx, MOM_VEC_CALLER, ma));
    TravArgs ta = trav_args(ctx, w);
    ta.order = 0;
    ta.momhi = nullptr;
    ta.src4 = ctx->va.p;
    ta.out = gradf;
    RETURN_IF(run_traverse(ctx, OP_G, TR_OUT_CALLER, ta));
    // p: sources g, each target with its own mu (sorted, kept in va)
    MomArgs mb = mom_args(ctx, w, true);
    mb.cs = g;
    mb.outs = ctx->rho.p;
    RETURN_IF(run_moments(ctx, MOM_SCALAR_CALLER, mb));
    TravArgs tb = trav_args(ctx, w);
    tb.order = 0;
    tb.momhi = nullptr;
    tb.srcs = ctx->rho.p;
    tb.tvec = ctx->va.p;
    tb.gc = g;
    tb.gradf = gradf;
    tb.out = dx_out;
    return run_traverse(ctx, OP_P, TR_POSGRAD, tb);
}

extern "C" {

wnnc_status wnnc_winding_grad_x(wnnc_ctx ctx, const float *n, const float *sigma, float w,
                                const float *g, float *dx_out) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    HIPCHK(ctx->gradf.ensure(3 * ctx->n));
    return winding_grad_x_impl(ctx, n, sigma, w, g, dx_out, ctx->gradf.p);
}

wnnc_status wnnc_winding_grad_x_noalloc(wnnc_ctx ctx, const float *n, const float *sigma,
                                        float w, const float *g, float *dx_out) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    if (ctx->n > kNoallocMaxPoints)
        return fail(WNNC_EINVAL, "wnnc_winding_grad_x_noalloc: %lld points exceed the limit of %lld",
                    (long long)ctx->n, (long long)kNoallocMaxPoints);
    float *scratch = noalloc_scratch(ctx->device);
    if (!scratch) return fail(WNNC_EDEVICE, "no scratch address for device %d", ctx->device);
    // timing creates events: this entry point runs untimed
    const unsigned saved = ctx->flags;
    ctx->flags &= ~(WNNC_FLAG_TIME_KERNELS | WNNC_FLAG_TIME_TRAVERSAL);
    const wnnc_status s = winding_grad_x_impl(ctx, n, sigma, w, g, dx_out, scratch);
    ctx->flags = saved;
    return s;
}

wnnc_status wnnc_gradient_grad_x(wnnc_ctx ctx, const float *n, const float *sigma, float w,
                                 const float *v, float *dx_out) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    if (!n || !v || !dx_out) return fail(WNNC_EINVAL, "null pointer");
    if (!finite_nonneg(w)) return fail(WNNC_EINVAL, "w must be finite and >= 0");
    RETURN_IF(check_finite(ctx, n, 3 * ctx->n, "n"));
    RETURN_IF(check_finite(ctx, sigma, ctx->n, "sigma"));
    RETURN_IF(check_finite(ctx, v, 3 * ctx->n, "v"));
    const int64_t N = ctx->n;
    hipStream_t st = ctx->stream;
    HIPCHK(ctx->gradf.ensure(3 * N));
    // v in sorted order (vb); mu in sorted order with its representatives (va)
    HIPCHK(launch_gather_vec(v, ctx->perm.p, ctx->vb.p, N, st));
    MomArgs ma = mom_args(ctx, w, true);
    ma.cn = n;
    ma.csig = sigma;
    ma.out4 = ctx->va.p;
    RETURN_IF(run_moments(ctx, MOM_VEC_CALLER, ma));
    // T(mu; v): sources mu, each target with its v -> gradf (caller order)
    TravArgs ta = trav_args(ctx, w);
    ta.order = 0;
    ta.momhi = nullptr;
    ta.src4 = ctx->va.p;
    ta.tvec = ctx->vb.p;
    ta.out = ctx->gradf.p;
    RETURN_IF(run_traverse(ctx, OP_T, TR_OUT_CALLER, ta));
    // T(v; mu): sources v, each target with its mu, added to the first
    MomArgs mb = mom_args(ctx, w, true);
    mb.src4 = ctx->vb.p;
    RETURN_IF(run_moments(ctx, MOM_VEC_SORTED, mb));
    TravArgs tb = trav_args(ctx, w);
    tb.order = 0;
    tb.momhi = nullptr;
    tb.src4 = ctx->vb.p;
    tb.tvec = ctx->va.p;
    tb.gradf = ctx->gradf.p;
    tb.out = dx_out;
    return run_traverse(ctx, OP_T, TR_ACCUM, tb);
}

wnnc_status wnnc_adjoint(wnnc_ctx ctx, const float *s, float w, float *out) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    if (!s || !out) return fail(WNNC_EINVAL, "null pointer");
    if (!finite_nonneg(w)) return fail(WNNC_EINVAL, "w must be finite and >= 0");
    RETURN_IF(check_finite(ctx, s, ctx->n, "s"));
    MomArgs ma = mom_args(ctx, w);
    ma.cs = s;
    ma.outs = ctx->rho.p;
    RETURN_IF(run_moments(ctx, MOM_SCALAR_CALLER, ma));
    TravArgs ta = trav_args(ctx, w);
    ta.srcs = ctx->rho.p;
    ta.out = out;
    return run_traverse(ctx, OP_AT, TR_OUT_CALLER, ta);
}

wnnc_status wnnc_energy(wnnc_ctx ctx, const float *mu, float w, double gscale, double *E_out,
                        float *grad_out) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    if (!mu) return fail(WNNC_EINVAL, "null mu");
    if (!finite_nonneg(w)) return fail(WNNC_EINVAL, "w must be finite and >= 0");
    if (!isfinite(gscale)) return fail(WNNC_EINVAL, "gscale must be finite");
    RETURN_IF(check_finite(ctx, mu, 3 * ctx->n, "mu"));
    if (!E_out && !grad_out) return WNNC_OK;
    hipStream_t st = ctx->stream;
    // rho = 1/2 - A mu (sorted), with per-group partial sums of rho^2
    MomArgs ma = mom_args(ctx, w);
    ma.cn = mu;
    ma.out4 = ctx->va.p;
    RETURN_IF(run_moments(ctx, MOM_VEC_CALLER, ma));
    TravArgs ta = trav_args(ctx, w);
    ta.src4 = ctx->va.p;
    ta.rho = ctx->rho.p;
    ta.partial = ctx->partial.p;
    RETURN_IF(run_traverse(ctx, OP_A, TR_RHO, ta));
    if (grad_out) {
        // gscale dE/dmu = -2 gscale A^T rho, in caller order
        MomArgs mb = mom_args(ctx, w);
        mb.srcs = ctx->rho.p;
        RETURN_IF(run_moments(ctx, MOM_SCALAR_SORTED, mb));
        TravArgs tb = trav_args(ctx, w);
        tb.srcs = ctx->rho.p;
        tb.out = grad_out;
        tb.oscale = -2.0 * gscale;
        RETURN_IF(run_traverse(ctx, OP_AT, TR_OUT_CALLER, tb));
    }
    if (E_out) {
        HIPCHK(ctx->scalars.ensure(ctx->nclouds + 1));
        double *dE = ctx->scalars.p + ctx->nclouds;
        HIPCHK(launch_sum_partials(ctx->partial.p, ctx->ngroups, dE, st));
        HIPCHK(hipMemcpyAsync(E_out, dE, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    return WNNC_OK;
}

// Iterations start..stop of Alg. 3 (schedule over iters) on the sorted mu in
// ctx->va.  zero: mu is 0 at the start (the first A(mu) is skipped).
// flips (device, per cloud, may be null): in the last iteration, the number
// of points whose WNNC update points against mu + alpha r.
// Width of iteration i of n (1-based) under schedule `sched`
// (wnnc_orient_opts; FP64 on the host, rounded once to FP32).
static double schedule_width(int sched, int i, int n, float w1, float w2) {
    if (n <= 1) return (double)w1;
    const double t = (double)(i - 1) / (n - 1);
    if (sched == WNNC_SCHEDULE_COSINE)
        return (double)w1 + ((double)w2 - (double)w1) * (1.0 + cos(M_PI * t)) / 2.0;
    if (sched == WNNC_SCHEDULE_EXPONENTIAL) return (double)w2 * pow((double)w1 / (double)w2, t);
    return (double)w2 * (n - i) / (n - 1) + (double)w1 * (i - 1) / (n - 1);
}

static wnnc_status run_iterations(wnnc_ctx ctx, int iters, float w1, float w2, int start, int stop,
                                  bool zero, unsigned long long *flips, int sched,
                                  const float *areas) {
    const int nt = ctx->ngroups;  // row stride of the per-group sums
    const int count = stop - start + 1;
    HIPCHK(ctx->energy.ensure((int64_t)count * ctx->nclouds));
    float4 *mu = ctx->va.p, *tmp = ctx->vb.p, *r = ctx->vr.p;
    float *rho = ctx->rho.p;
    // With the groups aligned to the moment pass's wavefronts, the moment
    // pass that reads a walk's output also runs that walk's combining pass
    // (one launch fewer); the G walk's is run by the next iteration's first
    // moment pass.
    const bool fuse_ok = ctx->gtab_ok && !(ctx->flags & WNNC_FLAG_SEPARATE_COMBINE);
    TravArgs pend_g;
    bool have_pend = false;
    for (int i = start; i <= stop; ++i) {
        const float wf = (float)schedule_width(sched, i, iters, w1, w2);
        double *erow = ctx->energy.p + (int64_t)(i - start) * ctx->nclouds;
        // gradient step (Alg. 2): rho = b - A mu, r = A^T rho, t = A r
        const bool first = zero && i == start;
        if (first) {
            // mu = 0: A mu = 0 exactly, so rho = 1/2 everywhere
            MomArgs ma = mom_args(ctx, wf);
            ma.outs = rho;
            RETURN_IF(run_moments(ctx, MOM_CONST_HALF, ma));
        } else {
            MomArgs ma = mom_args(ctx, wf);
            ma.src4 = mu;
            if (have_pend) {
                RETURN_IF(run_moments_comb(ctx, MOM_COMB_RESCALE, ma, OP_G, pend_g));
                have_pend = false;
            } else {
                RETURN_IF(run_moments(ctx, MOM_VEC_SORTED, ma));
            }
            TravArgs ta = trav_args(ctx, wf);
            ta.src4 = mu;
            ta.rho = rho;
            ta.partial = ctx->partial.p;
            MomArgs mb = mom_args(ctx, wf);
            mb.srcs = rho;
            const bool fuse = fuse_ok && mb.order == 0;
            RETURN_IF(run_traverse(ctx, OP_A, TR_RHO, ta, !fuse));
            if (fuse)
                RETURN_IF(run_moments_comb(ctx, MOM_COMB_RHO, mb, OP_A, ta));
            else
                RETURN_IF(run_moments(ctx, MOM_SCALAR_SORTED, mb));
        }
        {
            TravArgs ta = trav_args(ctx, wf);
            ta.srcs = rho;
            ta.out4 = r;
            ta.partial = ctx->partial.p + nt;
            MomArgs ma = mom_args(ctx, wf);
            ma.src4 = r;
            const bool fuse = fuse_ok && ma.order == 0;
            RETURN_IF(run_traverse(ctx, OP_AT, TR_R, ta, !fuse));
            if (fuse)
                RETURN_IF(run_moments_comb(ctx, MOM_COMB_R, ma, OP_AT, ta));
            else
                RETURN_IF(run_moments(ctx, MOM_VEC_SORTED, ma));
        }
        {
            TravArgs ta = trav_args(ctx, wf);
            ta.src4 = r;
            ta.partial = ctx->partial.p + 2 * nt;
            RETURN_IF(run_traverse(ctx, OP_A, TR_TSUM, ta));
        }
        HIPCHK(launch_alpha(ctx, first, erow));
        // mu <- mu + alpha r, then the WNNC update and rescale
        {
            MomArgs ma = mom_args(ctx, wf);
            ma.src4 = mu;
            ma.r4 = r;
            ma.out4 = tmp;
            RETURN_IF(run_moments(ctx, MOM_AXPY, ma));
            TravArgs ta = trav_args(ctx, wf);
            ta.src4 = tmp;
            ta.out4 = mu;
            ta.areas = areas;
            if (i == stop) ta.flips = flips;
            // (the next iteration's first moment pass combines this walk)
            const bool fuse = i < stop && fuse_ok && mom_args(ctx, wf).order == 0;
            RETURN_IF(run_traverse(ctx, OP_G, TR_RESCALE, ta, !fuse));
            if (fuse) {
                pend_g = ta;
                have_pend = true;
            }
        }
    }
    ctx->last_energy_count = count;
    return WNNC_OK;
}

wnnc_status wnnc_orient_preset(int preset, wnnc_orient_opts *out) {
    if (!out) return fail(WNNC_EINVAL, "null out");
    wnnc_orient_opts o = {40, 0.002f, 0.016f, 1, 0, WNNC_SCHEDULE_LINEAR, nullptr};
    switch (preset) {
    case WNNC_PRESET_DEFAULT: break;
    case WNNC_PRESET_NOISE_025: o.w1 = 0.02f, o.w2 = 0.08f; break;
    case WNNC_PRESET_NOISE_05: o.w1 = 0.03f, o.w2 = 0.12f; break;
    case WNNC_PRESET_NOISE_1: o.w1 = 0.04f, o.w2 = 0.16f; break;
    case WNNC_PRESET_SCAN: o.w1 = 0.01f, o.w2 = 0.04f; break;
    case WNNC_PRESET_HIGH_GENUS: o.iters = 300; break;
    default: return fail(WNNC_EINVAL, "unknown preset %d", preset);
    }
    *out = o;
    return WNNC_OK;
}

wnnc_status wnnc_orient(wnnc_ctx ctx, const wnnc_orient_opts *opts, const float *mu0,
                        float *mu_out) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    if (!mu_out) return fail(WNNC_EINVAL, "null mu_out");
    wnnc_orient_opts o = {40, 0.002f, 0.016f, 1, 0, WNNC_SCHEDULE_LINEAR, nullptr};
    if (opts) o = *opts;
    if (o.iters < 1) return fail(WNNC_EINVAL, "iters must be >= 1");
    if (o.schedule < WNNC_SCHEDULE_LINEAR || o.schedule > WNNC_SCHEDULE_EXPONENTIAL)
        return fail(WNNC_EINVAL, "unknown width schedule %d", o.schedule);
    if (o.schedule == WNNC_SCHEDULE_EXPONENTIAL && !(o.w1 > 0.0f && o.w2 > 0.0f))
        return fail(WNNC_EINVAL, "the exponential schedule needs w1, w2 > 0");
    if (o.start_iter < 1 || o.start_iter > o.iters)
        return fail(WNNC_EINVAL, "start_iter must be in 1..iters");
    const int stop = o.stop_iter == 0 ? o.iters : o.stop_iter;
    if (stop < o.start_iter || stop > o.iters)
        return fail(WNNC_EINVAL, "stop_iter must be 0 or in start_iter..iters");
    if (!finite_nonneg(o.w1) || !finite_nonneg(o.w2))
        return fail(WNNC_EINVAL, "widths must be finite and >= 0");
    RETURN_IF(check_finite(ctx, mu0, 3 * ctx->n, "mu0"));
    RETURN_IF(check_finite(ctx, o.areas, ctx->n, "areas"));
    const int64_t N = ctx->n;
    hipStream_t st = ctx->stream;
    const bool zero = mu0 == nullptr;
    if (zero)
        HIPCHK(launch_zero_f4(ctx->va.p, N, st));
    else
        HIPCHK(launch_gather_vec(mu0, ctx->perm.p, ctx->va.p, N, st));
    const float *areas = nullptr;
    if (o.areas) {
        HIPCHK(ctx->areas.ensure(N));
        HIPCHK(launch_gather_scalar(o.areas, ctx->perm.p, ctx->areas.p, N, st));
        areas = ctx->areas.p;
    }
    RETURN_IF(run_iterations(ctx, o.iters, o.w1, o.w2, o.start_iter, stop, zero, nullptr,
                             o.schedule, areas));
    HIPCHK(launch_scatter_vec(ctx->va.p, ctx->perm.p, mu_out, N, st));
    return WNNC_OK;
}

wnnc_status wnnc_warm_orient(wnnc_ctx ctx, const float *params, const wnnc_warm_opts *opts,
                             float *mu_out, wnnc_warm_report *report) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    if (!params || !mu_out) return fail(WNNC_EINVAL, "null pointer");
    RETURN_IF(check_finite(ctx, params, kMlpParams, "params"));
    wnnc_warm_opts o = {6, 0.002f, 0.016f, 0.005f, 40, 0.016f, 0.4f, 0, 0.0f};
    if (opts) o = *opts;
    if (o.iters < 1 || o.fallback_iters < 1) return fail(WNNC_EINVAL, "iteration counts must be >= 1");
    if (o.max_iters < 0 || o.max_iters > 100000) return fail(WNNC_EINVAL, "max_iters out of range");
    if (!(o.stop_frac >= 0.0f && o.stop_frac <= 1.0f))
        return fail(WNNC_EINVAL, "stop_frac must be in [0, 1]");
    if (!finite_nonneg(o.w1) || !finite_nonneg(o.w2) || !finite_nonneg(o.fallback_w2))
        return fail(WNNC_EINVAL, "widths must be finite and >= 0");
    if (!(o.max_disagree >= 0.0f && o.max_disagree <= 1.0f))
        return fail(WNNC_EINVAL, "max_disagree must be in [0, 1]");
    if (!(o.max_pred_disagree >= 0.0f && o.max_pred_disagree <= 1.0f))
        return fail(WNNC_EINVAL, "max_pred_disagree must be in [0, 1]");
    const int64_t N = ctx->n;
    const int B = ctx->nclouds;
    hipStream_t st = ctx->stream;
    // 1. predicted unit normals (caller order, in vr reinterpreted as N*3)
    HIPCHK(ctx->feat.ensure(N * kMlpIn));
    HIPCHK(ctx->mlp_y.ensure(N * kMlpOut));
    HIPCHK(ctx->nhat.ensure(N * 3));
    HIPCHK(launch_knn_features(ctx, ctx->feat.p, nullptr));
    HIPCHK(mlp_forward(ctx, params, ctx->feat.p, N, ctx->mlp_y.p));
    HIPCHK(mlp_normals(ctx, ctx->mlp_y.p, N, ctx->nhat.p));
    // 2. per-cloud least-squares scale beta = <A n, 1/2> / |A n|^2 at the
    //    first width of the warm schedule; mu0 = beta n
    {
        MomArgs ma = mom_args(ctx, o.iters > 1 ? o.w2 : o.w1);
        ma.cn = ctx->nhat.p;
        ma.out4 = ctx->vb.p;
        RETURN_IF(run_moments(ctx, MOM_VEC_CALLER, ma));
        TravArgs ta = trav_args(ctx, o.iters > 1 ? o.w2 : o.w1);
        ta.src4 = ctx->vb.p;
        ta.partial = ctx->partial.p;
        RETURN_IF(run_traverse(ctx, OP_A, TR_SCALE, ta));
        HIPCHK(launch_warm_scale(ctx, ctx->vb.p, ctx->va.p));
    }
    // 3. short schedule from mu0; self-checks: the last update against mu
    //    (flip_ctr[0..B)) and the result against the prediction
    //    (flip_ctr[B..2B))
    HIPCHK(ctx->flip_ctr.ensure(2 * B));
    HIPCHK(hipMemsetAsync(ctx->flip_ctr.p, 0, (size_t)(2 * B) * sizeof(unsigned long long), st));
    RETURN_IF(run_iterations(ctx, o.iters, o.w1, o.w2, 1, o.iters, false, ctx->flip_ctr.p,
                             WNNC_SCHEDULE_LINEAR, nullptr));
    std::vector<unsigned long long> fl((size_t)(2 * B));
    // the worst per-cloud fraction of the counters at `base`
    auto worst_of = [&](int base) {
        double wv = 0.0;
        for (int c = 0; c < B; ++c)
            wv = std::max(wv, (double)fl[base + c] / (double)(ctx->offsets[c + 1] - ctx->offsets[c]));
        return wv;
    };
    int ran = o.iters;
    // until convergence: one more iteration at w1 while an update still
    // turns more than stop_frac of some cloud's points and fewer than the
    // update before (at a fixed width the sign changes need not vanish:
    // points can keep turning back and forth)
    double prev = HUGE_VAL;
    while (o.max_iters > ran) {
        HIPCHK(hipMemcpyAsync(fl.data(), ctx->flip_ctr.p, (size_t)B * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const double cur = worst_of(0);
        if (cur <= (double)o.stop_frac || cur >= prev) break;
        prev = cur;
        HIPCHK(hipMemsetAsync(ctx->flip_ctr.p, 0, (size_t)B * sizeof(unsigned long long), st));
        RETURN_IF(run_iterations(ctx, 1, o.w1, o.w1, 1, 1, false, ctx->flip_ctr.p,
                                 WNNC_SCHEDULE_LINEAR, nullptr));
        ++ran;
    }
    HIPCHK(launch_pred_disagree(ctx, ctx->va.p, ctx->nhat.p, ctx->flip_ctr.p + B));
    HIPCHK(hipMemcpyAsync(fl.data(), ctx->flip_ctr.p, (size_t)(2 * B) * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double worst = worst_of(0), worst_pred = worst_of(B);
    const bool fallback =
        worst > (double)o.max_disagree || worst_pred > (double)o.max_pred_disagree;
    // 4. the plain method when the check fails
    if (fallback) {
        HIPCHK(launch_zero_f4(ctx->va.p, N, st));
        RETURN_IF(run_iterations(ctx, o.fallback_iters, o.w1, o.fallback_w2, 1, o.fallback_iters,
                                 true, nullptr, WNNC_SCHEDULE_LINEAR, nullptr));
    }
    HIPCHK(launch_scatter_vec(ctx->va.p, ctx->perm.p, mu_out, N, st));
    if (report) {
        report->iterations = ran + (fallback ? o.fallback_iters : 0);
        report->fallback = fallback ? 1 : 0;
        report->max_disagree = worst;
        report->max_pred_disagree = worst_pred;
    }
    return WNNC_OK;
}

wnnc_status wnnc_normals(wnnc_ctx ctx, const float *mu, int64_t N, double scale, float *n_out,
                         float *area_out) {
    CHECK_CTX(ctx);
    if (!mu || !n_out) return fail(WNNC_EINVAL, "null pointer");
    if (N < 1 || N > INT32_MAX) return fail(WNNC_EINVAL, "N = %lld out of range", (long long)N);
    if (!(isfinite(scale) && scale > 0.0)) return fail(WNNC_EINVAL, "scale must be finite and > 0");
    HIPCHK(launch_normals(mu, N, scale, n_out, area_out, ctx->stream));
    return WNNC_OK;
}

wnnc_status wnnc_knn_features(wnnc_ctx ctx, float *feat_out, int32_t *nbr_out) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    if (!feat_out) return fail(WNNC_EINVAL, "null feat_out");
    HIPCHK(launch_knn_features(ctx, feat_out, nbr_out));
    return WNNC_OK;
}

wnnc_status wnnc_knn_areas(wnnc_ctx ctx, int k, float *areas_out) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    if (!areas_out) return fail(WNNC_EINVAL, "null areas_out");
    if (k < 2 || k > 16) return fail(WNNC_EINVAL, "k = %d out of range 2..16", k);
    HIPCHK(launch_knn(ctx));
    HIPCHK(launch_knn_areas(ctx, k, areas_out));
    return WNNC_OK;
}

wnnc_status wnnc_mlp_forward(wnnc_ctx ctx, const float *params, const float *feat, int64_t N,
                             float *normals_out) {
    CHECK_CTX(ctx);
    if (!params || !feat || !normals_out) return fail(WNNC_EINVAL, "null pointer");
    if (N < 1 || N > INT32_MAX) return fail(WNNC_EINVAL, "N = %lld out of range", (long long)N);
    HIPCHK(ctx->mlp_y.ensure(N * kMlpOut));
    HIPCHK(mlp_forward(ctx, params, feat, N, ctx->mlp_y.p));
    HIPCHK(mlp_normals(ctx, ctx->mlp_y.p, N, normals_out));
    return WNNC_OK;
}

wnnc_status wnnc_mlp_grad(wnnc_ctx ctx, const float *params, const float *feat,
                          const float *labels, int64_t N, float *grad_out, double *loss_out) {
    CHECK_CTX(ctx);
    if (!params || !feat || !labels || !grad_out) return fail(WNNC_EINVAL, "null pointer");
    if (N < 1 || N > INT32_MAX) return fail(WNNC_EINVAL, "N = %lld out of range", (long long)N);
    HIPCHK(mlp_loss_grad(ctx, params, feat, labels, N, grad_out, loss_out));
    return WNNC_OK;
}

wnnc_status wnnc_mlp_adam(wnnc_ctx ctx, float *params, float *m, float *v, const float *grad,
                          int step, float lr, float beta1, float beta2, float eps) {
    CHECK_CTX(ctx);
    if (!params || !m || !v || !grad) return fail(WNNC_EINVAL, "null pointer");
    if (step < 1) return fail(WNNC_EINVAL, "step must be >= 1");
    if (!(lr > 0.f && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
        return fail(WNNC_EINVAL, "bad Adam hyperparameters");
    HIPCHK(mlp_adam(ctx, params, m, v, grad, step, lr, beta1, beta2, eps));
    return WNNC_OK;
}

wnnc_status wnnc_orient_energy(wnnc_ctx ctx, double *host_out, int count) {
    CHECK_CTX(ctx);
    if (!host_out || count < 0) return fail(WNNC_EINVAL, "bad output");
    if (count > ctx->last_energy_count)
        return fail(WNNC_EINVAL, "only %d energies recorded", ctx->last_energy_count);
    if (count == 0) return WNNC_OK;
    HIPCHK(hipMemcpyAsync(host_out, ctx->energy.p, (size_t)count * ctx->nclouds * sizeof(double),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return WNNC_OK;
}

wnnc_status wnnc_stats(wnnc_ctx ctx, wnnc_stats_t *out) {
    CHECK_CTX(ctx);
    if (!out) return fail(WNNC_EINVAL, "null output");
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (auto &t : ctx->pending) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, t.a, t.b));
        if (t.kind < kKindMoments)
            ctx->trav_ms[t.kind] += ms;
        else if (t.kind == kKindMoments)
            ctx->mom_ms += ms;
        else
            ctx->comb_ms += ms;
        ctx->event_pool.push_back(t.a);
        ctx->event_pool.push_back(t.b);
    }
    ctx->pending.clear();
    memset(out, 0, sizeof(*out));
    out->n_points = ctx->built ? ctx->n : 0;
    out->n_nodes = ctx->built ? ctx->m : 0;
    unsigned long long pc[kOpKinds] = {};
    if (ctx->pair_ctr.p) {
        HIPCHK(hipMemcpy(pc, ctx->pair_ctr.p, sizeof(pc), hipMemcpyDeviceToHost));
    }
    for (int k = 0; k < kOpKinds; ++k) {
        out->calls[k] = ctx->calls[k];
        out->pairs[k] = (int64_t)pc[k];
        out->traverse_ms[k] = ctx->trav_ms[k];
    }
    out->moments_ms = ctx->mom_ms;
    out->combine_ms = ctx->comb_ms;
    out->build_ms = ctx->build_ms;
    out->n_clouds = ctx->built ? ctx->nclouds : 0;
    out->tile = ctx->tpl | (ctx->prefetch << 8) | ((int64_t)ctx->split << 16);
    out->n_groups = ctx->built ? ctx->ngroups : 0;
    out->n_tasks = ctx->built ? ctx->ntasks : 0;
    for (int k = 0; k < kOpKinds; ++k)
        if (prefetch_of(ctx, (Op)k)) out->prefetch_ops |= int64_t(1) << k;
    return WNNC_OK;
}

wnnc_status wnnc_reset_stats(wnnc_ctx ctx) {
    CHECK_CTX(ctx);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (auto &t : ctx->pending) {
        ctx->event_pool.push_back(t.a);
        ctx->event_pool.push_back(t.b);
    }
    ctx->pending.clear();
    for (int k = 0; k < kOpKinds; ++k) {
        ctx->calls[k] = 0;
        ctx->trav_ms[k] = 0;
    }
    ctx->mom_ms = 0;
    ctx->comb_ms = 0;
    HIPCHK(ctx->pair_ctr.ensure(kOpKinds));
    HIPCHK(hipMemsetAsync(ctx->pair_ctr.p, 0, kOpKinds * sizeof(unsigned long long), ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return WNNC_OK;
}

wnnc_status wnnc_tree_export(wnnc_ctx ctx, int32_t *depth, int32_t *leaf, int64_t *begin,
                             int64_t *end, int64_t *perm) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    std::vector<int4> topo((size_t)ctx->m);
    std::vector<uint32_t> pm((size_t)ctx->n);
    HIPCHK(hipMemcpyAsync(topo.data(), ctx->topo.p, (size_t)ctx->m * sizeof(int4),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(pm.data(), ctx->perm.p, (size_t)ctx->n * sizeof(uint32_t),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int64_t k = 0; k < ctx->m; ++k) {
        if (depth) depth[k] = topo_depth(topo[k].w);
        if (leaf) leaf[k] = topo_leaf(topo[k].w);
        if (begin) begin[k] = topo[k].y;
        if (end) end[k] = topo[k].z;
    }
    if (perm)
        for (int64_t i = 0; i < ctx->n; ++i) perm[i] = pm[i];
    return WNNC_OK;
}

wnnc_status wnnc_moments_export(wnnc_ctx ctx, const float *nu, int dim, float *xB, float *nuB,
                                float *W) {
    CHECK_CTX(ctx);
    CHECK_BUILT(ctx);
    if (!nu) return fail(WNNC_EINVAL, "null nu");
    if (dim != 1 && dim != 3) return fail(WNNC_EINVAL, "dim must be 1 or 3");
    HIPCHK(ctx->wbuf.ensure(ctx->m));
    MomArgs ma = mom_args(ctx, 0.0f);
    ma.wout = ctx->wbuf.p;
    if (dim == 3) {
        ma.cn = nu;
        ma.out4 = ctx->vb.p;
        RETURN_IF(run_moments(ctx, MOM_VEC_CALLER, ma));
    } else {
        ma.cs = nu;
        ma.outs = ctx->rho.p;
        RETURN_IF(run_moments(ctx, MOM_SCALAR_CALLER, ma));
    }
    std::vector<float4> mom((size_t)(kRecStride * ctx->m));
    std::vector<float> wv((size_t)ctx->m);
    HIPCHK(hipMemcpyAsync(mom.data(), ctx->mom.p, (size_t)(kRecStride * ctx->m) * sizeof(float4),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(wv.data(), ctx->wbuf.p, (size_t)ctx->m * sizeof(float),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int64_t k = 0; k < ctx->m; ++k) {
        const float4 p = mom[kRecStride * k], v = mom[kRecStride * k + 1];
        const float4 lo = mom[kRecStride * k + 2];
        if (xB) {
            xB[3 * k] = (float)((double)p.x + (double)lo.x);
            xB[3 * k + 1] = (float)((double)p.y + (double)lo.y);
            xB[3 * k + 2] = (float)((double)p.z + (double)lo.z);
        }
        if (W) W[k] = wv[k];
        if (nuB) {
            if (dim == 3) {
                nuB[3 * k] = v.x;
                nuB[3 * k + 1] = v.y;
                nuB[3 * k + 2] = v.z;
            } else {
                nuB[k] = v.x;
            }
        }
    }
    return WNNC_OK;
}

}  // extern "C"
