// Host-side entry points shared between the library's translation units.
#pragma once

#include <hip/hip_ext.h>

#include <tuple>
#include <utility>

#include "common.h"

namespace wnnc {

template <typename Tup, size_t... I>
inline hipError_t launch_packed(wnnc_ctx_s::LaunchEvents &ev, bool last, const void *k, dim3 grid,
                                dim3 block, hipStream_t st, Tup &vals, std::index_sequence<I...>) {
    void *argv[] = {(void *)&std::get<I>(vals)...};
    if (!ev.start) return hipLaunchKernel(k, grid, block, argv, 0, st);
    // a timed call: the kernel's own dispatch records the events, so that
    // timing adds no marker commands (and no idle gaps) to the stream
    hipEvent_t a = ev.started ? nullptr : ev.start, b = last ? ev.stop : nullptr;
    const hipError_t e = hipExtLaunchKernel(k, grid, block, argv, 0, st, a, b, 0);
    if (e == hipSuccess) {
        ev.started = true;
        ev.stopped = ev.stopped || last;
    }
    return e;
}

// Launches `kernel` (no dynamic LDS) on st, carrying the events of the timed
// call in progress: the start event on the call's first launch, the stop
// event on the launch marked `last`.
template <typename... KArgs, typename... Args>
inline hipError_t launch_k(wnnc_ctx_s::LaunchEvents &ev, bool last, void (*kernel)(KArgs...),
                           dim3 grid, dim3 block, hipStream_t st, Args... args) {
    static_assert(sizeof...(KArgs) == sizeof...(Args), "kernel argument count");
    std::tuple<KArgs...> vals{args...};
    return launch_packed(ev, last, (const void *)kernel, grid, block, st, vals,
                         std::index_sequence_for<KArgs...>{});
}

// Returns a HIP error from the enclosing function (host code).
#define TRY(x)                           \
    do {                                 \
        hipError_t _e = (x);             \
        if (_e != hipSuccess) return _e; \
    } while (0)

int64_t scan_tmp_size(int64_t n);
hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp,
                              hipStream_t st);

// Tree build steps (tree.hip).
// Normalizes each cloud (rows d_off[c]..d_off[c+1]) of P into P_norm; tmp
// holds normalize_tmp_doubles(nclouds) doubles.  Returns the offset in tmp
// of the per-cloud (centre x, y, z, scale) quadruples.
int64_t launch_normalize(const float *P, int64_t n, const int64_t *d_off, int nclouds,
                         float *P_norm, double *tmp, hipStream_t st);
int64_t normalize_tmp_doubles(int64_t nclouds);
hipError_t build_tree(wnnc_ctx_s *ctx, const float *P);
// Sorts M caller-order query points (M,3) by Morton key into ctx->qpts, with
// their caller rows in ctx->qperm.
hipError_t sort_queries(wnnc_ctx_s *ctx, const float *Q, int64_t M);
// Wavefront tasks for tile shape tpl and split size `split` (node visits per
// part, 0 = whole walks; used only with tpl = 1 and a recorded plan).
hipError_t make_tasks(wnnc_ctx_s *ctx, int tpl, int split);

// Moment pass (moments.hip): two launches, chunk pass then straddler pass.
hipError_t launch_moments(wnnc_ctx_s *ctx, MomMode mode, const MomArgs &a);
// A moment pass (MOM_COMB_*) whose chunk pass also runs the combining pass
// of the walk ta just launched without it (needs a.gtab: every cloud starts
// at a multiple of 64 points, one group per wavefront).
hipError_t launch_moments_comb(wnnc_ctx_s *ctx, MomMode mode, const MomArgs &a,
                               const TravArgs &ta);

// Traversal (traverse.hip).
// The walk kernel, then (when walks are split) the combining pass that adds
// the parts and runs the epilogue; launch_traverse_all issues both.
hipError_t launch_traverse(wnnc_ctx_s *ctx, Op op, TravMode mode, bool count, const TravArgs &a);
hipError_t launch_combine(wnnc_ctx_s *ctx, Op op, TravMode mode, const TravArgs &a);
inline hipError_t launch_traverse_all(wnnc_ctx_s *ctx, Op op, TravMode mode, bool count,
                                      const TravArgs &a) {
    const hipError_t e = launch_traverse(ctx, op, mode, count, a);
    return e != hipSuccess ? e : launch_combine(ctx, op, mode, a);
}
int trav_blocks(int64_t ntasks);
// Records the walk of every 64-target group (ctx->plan) for split planning;
// the tasks must be whole walks of single 64-target groups.
hipError_t record_plan(wnnc_ctx_s *ctx, const TravArgs &a);

// Glue (glue.hip).
// Step length per cloud from the per-group partial sums; first = the
// iteration started from mu = 0 (its energy is N_c / 4).  energy_row holds
// one entry per cloud.
hipError_t launch_alpha(wnnc_ctx_s *ctx, bool first, double *energy_row);
hipError_t launch_sum_partials(const double *partial, int n, double *out, hipStream_t st);
hipError_t launch_zero_f4(float4 *p, int64_t n, hipStream_t st);
hipError_t launch_gather_vec(const float *src, const uint32_t *perm, float4 *dst, int64_t n,
                             hipStream_t st);
// dst[i] = src[perm[i]] (caller order to sorted order)
hipError_t launch_check_finite(const float *a, int64_t n, uint32_t *flag, hipStream_t st);
hipError_t launch_gather_scalar(const float *src, const uint32_t *perm, float *dst, int64_t n,
                                hipStream_t st);
hipError_t launch_scatter_vec(const float4 *src, const uint32_t *perm, float *dst, int64_t n,
                              hipStream_t st);

hipError_t launch_normals(const float *mu, int64_t n, double scale, float *nrm, float *area,
                          hipStream_t st);

// Warm start (knn.hip, mlp.hip).
// k = 16 nearest neighbours of every point within its cloud (sorted
// indices, nearest first, -1 where missing) into ctx->knn_idx.
hipError_t launch_knn(wnnc_ctx_s *ctx);
hipError_t launch_knn_features(wnnc_ctx_s *ctx, float *feat, int32_t *nbr_caller);
// kNN local areas from ctx->knn_idx (launch_knn first), caller order.
hipError_t launch_knn_areas(wnnc_ctx_s *ctx, int k, float *areas_out);
hipError_t mlp_forward(wnnc_ctx_s *ctx, const float *P, const float *X, int64_t n, float *Y);
hipError_t mlp_normals(wnnc_ctx_s *ctx, const float *Y, int64_t n, float *out);
hipError_t mlp_loss_grad(wnnc_ctx_s *ctx, const float *P, const float *X, const float *L,
                         int64_t n, float *grad, double *loss);
// mu0[i] = beta_c n[i] (sorted) with beta_c = (1/2) sum s / sum s^2 over
// cloud c from the TR_SCALE partials.
hipError_t launch_warm_scale(wnnc_ctx_s *ctx, const float4 *n_sorted, float4 *mu0);
// count[c] += points of cloud c whose sorted mu points against the caller-
// order prediction nhat (N,3).
hipError_t launch_pred_disagree(wnnc_ctx_s *ctx, const float4 *mu, const float *nhat,
                                unsigned long long *count);
hipError_t mlp_adam(wnnc_ctx_s *ctx, float *P, float *m, float *v, const float *g, int step,
                    float lr, float b1, float b2, float eps);

// Static scratch of the no-allocation entry points (noalloc.hip): at most
// kNoallocMaxPoints points.  noalloc_setup takes the array's address on
// `device` (which must be current), once per device; noalloc_scratch
// returns it (null before the set-up).
constexpr int64_t kNoallocMaxPoints = int64_t(1) << 20;
static_assert(kNoallocMaxPoints == WNNC_NOALLOC_MAX_POINTS, "no-allocation limit");
hipError_t noalloc_setup(int device);
float *noalloc_scratch(int device);

}  // namespace wnnc
