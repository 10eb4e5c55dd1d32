/*
 * wnnc.h -- C ABI of the MI355X WNNC library.
 *
 * The library evaluates, on one AMD Instinct MI355X (gfx950), the three
 * operators of WNNC normal orientation (Lin, Shi, Liu 2024) with the paper's
 * treecode, and runs the full WNNC iteration on the device:
 *
 *   winding number  s_i    = F(x_i; mu)  = sum_j gradPhi(x_i - x_j) . mu_j
 *                                                  (eq. wnf-discretization)
 *   gradient        grad F(x_i; mu)      = sum_j HPhi(x_i - x_j) mu_j
 *                                                  (Sec. 4.2; G = -grad F)
 *   adjoint         (A^T s)_j            = sum_i s_i gradPhi(x_i - x_j)
 *                                                  (Alg. 2)
 *   orientation     Alg. 3 (Alg. 2 gradient step, WNNC update, rescale)
 *
 * with gradPhi(y) = -y/(4 pi |y|^3) and HPhi(y) = -I/(4 pi |y|^3) +
 * 3 y y^T/(4 pi |y|^5); every pair closer than the smoothing width w (and
 * every coincident pair) contributes zero (Sec. 4.4).  mu_j = n_j sigma_j is
 * the oriented surface element: unit normal times area weight (Sec. 3).
 *
 * Treecode (Sec. 4.5, Alg. 4): an octree over [-1,1]^3 split while a node
 * holds more than one point and is shallower than the maximum depth D; per
 * call, nu-representatives x_B = sum |nu_i| x_i / sum |nu_i|, nu_B = sum nu_i;
 * per target, a node is replaced by its representative when
 * |x - x_B| > c * width(B), width(B) = 2^(1 - depth), otherwise its children
 * are visited (a leaf sums its points directly).  Nodes whose attributes are
 * all zero are skipped.
 *
 * Beyond the paper (each call documents its own definition): many clouds in
 * one forest (wnnc_build_batched), the winding number at query points
 * (wnnc_winding_at), a far field of higher order and a cutoff-safe
 * acceptance (wnnc_set_far_field), other width schedules and fixed areas
 * (wnnc_orient_opts), kNN local areas (wnnc_knn_areas), position gradients
 * (wnnc_winding_grad_x, wnnc_gradient_grad_x) and a learned warm start
 * (wnnc_warm_orient).
 *
 * Conventions
 * -----------
 * * Every float pointer is a DEVICE pointer to contiguous FP32 data owned by
 *   the caller; (N,3) arrays are row-major (x0,y0,z0,x1,...), in the caller's
 *   point order.  Host pointers are marked "host".
 * * Calls enqueue work on the context's stream and return without waiting,
 *   unless marked "synchronizes".  Outputs are valid once the stream has
 *   reached the call.  Inputs must stay valid until then.
 * * The context owns the octree, the point permutation and all scratch
 *   memory; wnnc_destroy frees them.  The caller owns every I/O buffer.
 * * A context is used by one host thread at a time.
 * * Errors: every call returns a wnnc_status; on failure wnnc_last_error()
 *   gives a message (thread-local, valid until the next failing call on the
 *   thread).  Invalid arguments return WNNC_EINVAL before any work is
 *   enqueued.  Non-finite inputs give unspecified (finite or not) results,
 *   unless WNNC_FLAG_CHECK_FINITE is set: then they return WNNC_ENUMERIC
 *   before any work is enqueued.
 */
#ifndef WNNC_H
#define WNNC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wnnc_ctx_s *wnnc_ctx;

typedef enum {
    WNNC_OK = 0,
    WNNC_EINVAL = -1,   /* bad argument (NULL, size, option range) */
    WNNC_ENOMEM = -2,   /* device allocation failed */
    WNNC_EDEVICE = -3,  /* a HIP runtime call or kernel launch failed */
    WNNC_ESTATE = -4,   /* no tree built yet (call wnnc_build first) */
    WNNC_ENUMERIC = -5, /* an input holds NaN or infinity (WNNC_FLAG_CHECK_FINITE) */
} wnnc_status;

/* Treecode options (Sec. 5.1.1 defaults in brackets). */
typedef struct {
    float c;        /* acceptance threshold c > 0 [2] */
    int max_depth;  /* maximum octree depth D, 1..15 [15] */
    int leaf_cap;   /* a node is split while it holds more than leaf_cap
                       points (and is shallower than D), 1..256 [1: the
                       paper's tree]; larger leaves are summed directly by
                       the targets that do not accept them (an extension) */
} wnnc_tree_opts;

/* Alg. 3 options (Sec. 5.1.1 defaults in brackets). */
typedef struct {
    int iters;       /* n >= 1 [40] */
    float w1, w2;    /* final and initial smoothing widths, normalized frame
                        [0.002, 0.016]; w = w2 (n-i)/(n-1) + w1 (i-1)/(n-1),
                        w = w1 when n = 1 */
    int start_iter;  /* first iteration index i, 1..n [1]; with mu0 this
                        resumes an interrupted run exactly */
    int stop_iter;   /* last iteration index run, start_iter..n, or 0 for n
                        [0]; (mu, i) is the whole state, so stopping at k and
                        resuming at k+1 with the returned mu reproduces an
                        uninterrupted run bit for bit */
    int schedule;    /* width schedule [WNNC_SCHEDULE_LINEAR, the above];
                        the variants named in Sec. 5.5.1, both from w2 at
                        i = 1 to w1 at i = n, t = (i-1)/(n-1):
                        COSINE w = w1 + (w2 - w1)(1 + cos(pi t))/2,
                        EXPONENTIAL w = w2 (w1/w2)^t (w1, w2 > 0) */
    const float *areas; /* NULL [the method], or (N) caller-order device
                        areas sigma_i >= 0 in the normalized frame: the
                        rescale of Alg. 3 becomes mu_i <- G_i sigma_i/|G_i|
                        (Sec. 6.1.1), so |mu_i| = sigma_i */
} wnnc_orient_opts;

#define WNNC_SCHEDULE_LINEAR 0
#define WNNC_SCHEDULE_COSINE 1
#define WNNC_SCHEDULE_EXPONENTIAL 2

/* Instrumentation flags (wnnc_set_flags). */
#define WNNC_FLAG_COUNT_PAIRS 1u  /* count pair evaluations (slower kernels) */
#define WNNC_FLAG_TIME_KERNELS 2u /* time every traversal, moment and
                                     combining launch with HIP events carried
                                     by the launches themselves */
#define WNNC_FLAG_CHECK_FINITE 4u /* check every float input array for NaN and
                                     infinity first (WNNC_ENUMERIC; each such
                                     call then synchronizes) */
#define WNNC_FLAG_TIME_TRAVERSAL 8u /* time the traversal launches only (fills
                                       traverse_ms; about a third of the
                                       timing overhead of WNNC_FLAG_TIME_KERNELS) */
#define WNNC_FLAG_SEPARATE_COMBINE 16u /* in Alg. 3's iterations, run the split
                                          walks' combining passes as launches of
                                          their own instead of inside the moment
                                          pass that reads their output (the same
                                          arithmetic, for checking; slower) */

/* Operator kinds, indices of the per-kind statistics. */
#define WNNC_OP_A 0
#define WNNC_OP_AT 1
#define WNNC_OP_G 2
#define WNNC_OP_P 3 /* the position-gradient walk of wnnc_winding_grad_x */
#define WNNC_OP_T 4 /* the position-gradient walks of wnnc_gradient_grad_x */

typedef struct {
    int64_t n_points;       /* N of the current tree */
    int64_t n_nodes;        /* octree nodes */
    int64_t calls[5];       /* operator applications per kind since reset */
    int64_t pairs[5];       /* pair evaluations per kind (WNNC_FLAG_COUNT_PAIRS):
                               accepted representatives plus points summed
                               directly, cut-off pairs included */
    double traverse_ms[5];  /* summed traversal-kernel time per kind
                               (WNNC_FLAG_TIME_KERNELS or
                               WNNC_FLAG_TIME_TRAVERSAL) */
    double moments_ms;      /* summed moment-pass time (WNNC_FLAG_TIME_KERNELS) */
    double build_ms;        /* last wnnc_build, device time (always timed) */
    int64_t n_clouds;       /* clouds in the current tree (1 for wnnc_build) */
    int64_t tile;           /* tile shape (wnnc_set_tile) | prefetch << 8 |
                               split (wnnc_set_split) << 16 */
    int64_t n_groups;       /* target groups (64 * tile shape targets) */
    int64_t n_tasks;        /* wavefronts per traversal launch (groups, or
                               parts of split walks) */
    double combine_ms;      /* summed time of the passes that add the parts of
                               split walks (WNNC_FLAG_TIME_KERNELS); not in
                               traverse_ms */
    int64_t prefetch_ops;   /* bit k set: operator kind k walks with prefetch
                               (wnnc_set_prefetch, or per kind by
                               wnnc_autotune) */
} wnnc_stats_t;

/* Create a context on HIP device `device`, enqueuing on `stream`
 * (a hipStream_t; NULL = the device's null stream).  Allocates nothing on
 * the device yet. */
wnnc_status wnnc_create(wnnc_ctx *out, int device, void *stream);

/* Free the context and every device buffer it owns.  Synchronizes. */
wnnc_status wnnc_destroy(wnnc_ctx ctx);

/* Change the stream later calls enqueue on. */
wnnc_status wnnc_set_stream(wnnc_ctx ctx, void *stream);

/* Instrumentation flags, see WNNC_FLAG_*. */
wnnc_status wnnc_set_flags(wnnc_ctx ctx, unsigned flags);

/* Sec. 5.1.1 normalization: centre the bounding box at the origin and scale
 * uniformly so that the largest half-extent is 10/11 ([-1,1]^3 with a margin
 * of 1/11).  P, P_norm: (N,3), may alias.  center_scale (host, 4 doubles):
 * centre x,y,z and scale s, so P_norm = (P - centre) * s computed in FP64
 * and rounded once.  Widths and areas are in the normalized frame
 * (areas scale by s^2).  Synchronizes. */
wnnc_status wnnc_normalize(wnnc_ctx ctx, const float *P, int64_t N, float *P_norm,
                           double *center_scale);

/* Batched normalization: B clouds stored one after another in P (cloud c =
 * rows offsets[c] .. offsets[c+1]-1; offsets is a host array of B+1
 * increasing values starting at 0, every cloud non-empty, 1 <= B <= 2^18),
 * each normalized on its own as in wnnc_normalize.  center_scale (host):
 * 4 doubles per cloud, or NULL.  Synchronizes. */
wnnc_status wnnc_normalize_batched(wnnc_ctx ctx, const float *P, const int64_t *offsets, int B,
                                   float *P_norm, double *center_scale);

/* Build the octree over normalized points P (N,3), 1 <= N < 2^31.  Points
 * outside [-1,1]^3 are clamped into the boundary cells.  Replaces any
 * previous tree.  opts NULL = paper defaults.  Synchronizes (reads back the
 * node count). */
wnnc_status wnnc_build(wnnc_ctx ctx, const float *P, int64_t N, const wnnc_tree_opts *opts);

/* Build one octree per cloud for B independent clouds (layout as in
 * wnnc_normalize_batched, each already normalized), as a single forest: one
 * sort orders the points cloud by cloud.  Every later call on the context
 * (operators, wnnc_orient) treats the clouds independently -- a point only
 * interacts with its own cloud -- while each operator is one launch over all
 * clouds.  Synchronizes. */
wnnc_status wnnc_build_batched(wnnc_ctx ctx, const float *P, const int64_t *offsets, int B,
                               const wnnc_tree_opts *opts);

/* Traversal tile shape: each wavefront serves tpl groups of 64 sorted
 * targets (tpl in {1, 2, 4}; default 1).  Results do not depend on it.
 * Synchronizes when a tree exists (rebuilds the task list). */
wnnc_status wnnc_set_tile(wnnc_ctx ctx, int tpl);
wnnc_status wnnc_get_tile(wnnc_ctx ctx, int *tpl);

/* Load balance of the traversal: with visits > 0 and tile shape 1, the
 * walk of a 64-target group that takes more than `visits` node visits (as
 * recorded by wnnc_build) runs as several wavefronts over consecutive
 * node ranges, each rebuilding its lanes' decisions at the range's
 * ancestors, and a combining pass adds their FP64 sums in range order.
 * The decisions and terms are those of the whole walk (Alg. 4); only the
 * FP64 summation order changes.  0 = whole walks; default 256.  visits in
 * 0..WNNC_MAX_SPLIT.  Synchronizes when a tree exists. */
#define WNNC_MAX_SPLIT (1 << 20)
wnnc_status wnnc_set_split(wnnc_ctx ctx, int visits);
wnnc_status wnnc_get_split(wnnc_ctx ctx, int *visits);

/* Deferred subtrees in the traversal: while a wavefront walks the tree for
 * its 64 targets in lockstep, a subtree that at most `lanes` of them need
 * (after their Alg. 4 decision to open its root) is set aside; the set-aside
 * (subtree, target) walks are then run packed across the lanes, each lane
 * walking one target's subtree on its own, so that lanes are not idle in
 * subtrees few targets need.  Every target makes the same decisions and
 * adds the same terms; only the order of the FP64 additions of its sum
 * changes.  Used with tile shape 1, the plain walk (prefetch off for the
 * operator) and Alg. 4's far field; otherwise ignored.  lanes in 0..64,
 * default 32; 0 walks every subtree in lockstep. */
wnnc_status wnnc_set_defer(wnnc_ctx ctx, int lanes);
wnnc_status wnnc_get_defer(wnnc_ctx ctx, int *lanes);

/* Software-pipelined node walk in the traversal: the skip successor's
 * record is loaded while the current node is visited (with the far field of
 * order > 0 the walk keeps plain loads).  Results do not depend on it, bit
 * for bit.  Default off; sets every operator kind (wnnc_autotune may then
 * choose per kind). */
wnnc_status wnnc_set_prefetch(wnnc_ctx ctx, int on);

/* Autotuner: times three iterations of Alg. 3 at width w from mu = 0 (the
 * fastest of two runs after a warm-up run) for each of
 * WNNC_AUTOTUNE_CONFIGS settings on the current tree, times the settings
 * within 3 % of the fastest again in turn (three rounds), and keeps the
 * fastest (a setting later in the list must be faster by more than 1 %):
 * (tpl, split) = (1, 0), (2, 0), (4, 0), (1, 1024), (1, 512), (1, 256),
 * (1, 128), (1, 64), each with prefetch off and on (in that order); the
 * short splits fill the chip on small clouds (few target groups).  times_out (host,
 * WNNC_AUTOTUNE_CONFIGS entries, may be NULL) receives the settings and
 * their times per iteration (the fastest run of each).  Then, on the chosen tiles, each operator
 * kind takes the other prefetch setting if its traversal launches are
 * faster with it by more than 1 % (see wnnc_stats_t.prefetch_ops).
 * Overwrites the context's iteration buffers; instrumentation statistics
 * are kept.  Synchronizes. */
#define WNNC_AUTOTUNE_CONFIGS 16
typedef struct {
    int tpl;
    int prefetch;
    int split;
    double ms;
} wnnc_tile_time;
wnnc_status wnnc_autotune(wnnc_ctx ctx, float w, wnnc_tile_time *times_out);

/* Winding number at the points: s_out[i] = F(x_i; mu), mu_j = n_j sigma_j.
 * n: (N,3); sigma: (N) or NULL (then n already holds mu); w >= 0. */
wnnc_status wnnc_winding(wnnc_ctx ctx, const float *n, const float *sigma, float w, float *s_out);

/* Winding number at query points anywhere in space (the field F of Sec. 3,
 * eq. of the winding number; e.g. on a grid, for the indicator function of
 * the oriented surface): s_out[k] = F(Q_k; mu), mu_j = n_j sigma_j over the
 * points of the built tree, which must be one cloud.  Q: (M,3) device, in
 * the frame of the points given to wnnc_build (normalized); M >= 1.  Each
 * query makes its own Alg. 4 decisions on the tree (c and D of the build),
 * with the cutoff w as for the points.  n, sigma, w as wnnc_winding.
 * Synchronizes.  EINVAL for a batched tree. */
wnnc_status wnnc_winding_at(wnnc_ctx ctx, const float *n, const float *sigma, float w,
                            const float *Q, int64_t M, float *s_out);

/* Gradient of the winding number at the points: grad_out (N,3) =
 * grad F(x_i; mu) = -G(mu)_i.  Arguments as wnnc_winding. */
wnnc_status wnnc_gradient(wnnc_ctx ctx, const float *n, const float *sigma, float w,
                          float *grad_out);

/* Adjoint of the winding-number operator applied to s (N): out (N,3),
 * out_j = sum_i s_i gradPhi(x_i - x_j) (with the treecode, using the
 * |s|-weighted representatives). */
wnnc_status wnnc_adjoint(wnnc_ctx ctx, const float *s, float w, float *out);

/* The energy that the gradient step of Alg. 2 descends (Sec. 4.3),
 * E(mu) = ||A_w mu - b||^2 with b_i = 1/2 (the winding number of the
 * surface points), and, optionally, its gradient: with rho = b - A_w mu and
 * r = A_w^T rho (the r of Alg. 2), dE/dmu = -2 r.
 * mu (N,3) device, caller order.  E_out (host, may be NULL): E, the FP64 sum
 * over every point of the tree (all clouds of a batched tree) of the FP32
 * rho_i^2, as in the iteration.  grad_out ((N,3) device, caller order, may
 * be NULL): gscale * dE/dmu = -2 gscale r (gscale the caller's chain-rule
 * factor, 1 for dE/dmu itself).  The treecode A^T is used as the adjoint
 * (with the treecode it is the gradient of E up to the treecode's
 * approximation error).  Synchronizes when E_out is given. */
wnnc_status wnnc_energy(wnnc_ctx ctx, const float *mu, float w, double gscale, double *E_out,
                        float *grad_out);

/* Gradient of L = sum_i g_i s_i, s = A_w(mu) (wnnc_winding), with respect to
 * the point positions (an extension: differentiable winding numbers in the
 * points).  Differentiating each pair term of A in both of its end points
 * (the cutoff held fixed) gives
 *   dL/dx_k = g_k grad F(x_k; mu) + p_k,
 *   p_k = -sum_i g_i HPhi(x_k - x_i) mu_k,
 * where p is one more treecode walk: scalar sources g (|g|-weighted
 * representatives, Alg. 4's acceptance) and, at each target, the target's
 * own mu_k.  mu (N,3) or n (N,3) with sigma (N) as in wnnc_winding, g (N),
 * dx_out (N,3): device, caller order, with respect to the normalized
 * points (multiply by the normalization scale s for the input points, since
 * x_norm = (x - centre) s).  Both walks
 * use Alg. 4's far field (order 0, without the cutoff-safe test) whatever
 * wnnc_set_far_field says. */
wnnc_status wnnc_winding_grad_x(wnnc_ctx ctx, const float *n, const float *sigma, float w,
                                const float *g, float *dx_out);

/* wnnc_winding_grad_x for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same result, bit for bit, with the
 * N x 3 grad F scratch in a static device array of the library instead of
 * context memory.  The call allocates nothing (no hipMalloc, hipFree or
 * event creation: timing flags are ignored for it); the tree and every
 * other buffer come from the last wnnc_build.  N (the built tree's point
 * count) <= WNNC_NOALLOC_MAX_POINTS, else WNNC_EINVAL before any work.  The
 * array (12 MiB) is held on every GPU the library runs on until the
 * process ends and is shared by all contexts on that GPU: calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * serialized by the caller.  Arguments as wnnc_winding_grad_x. */
#define WNNC_NOALLOC_MAX_POINTS (1 << 20)
wnnc_status wnnc_winding_grad_x_noalloc(wnnc_ctx ctx, const float *n, const float *sigma,
                                        float w, const float *g, float *dx_out);

/* Gradient of L = sum_i v_i . grad F(x_i; mu) (wnnc_gradient) with respect to
 * the point positions (an extension).  With the third-derivative tensor
 * T3Phi of Phi, differentiating each pair term of grad F in both end points
 * (the cutoff held fixed) gives
 *   dL/dx_k = sum_j T3Phi(x_k - x_j)[v_k, mu_j] + sum_i T3Phi(x_k - x_i)[mu_k, v_i],
 * two treecode walks of one kernel (vector sources, each target with its own
 * vector): sources mu with targets' v, then sources v with targets' mu.
 * n (N,3) with sigma (N) or NULL as in wnnc_gradient, v (N,3), dx_out (N,3):
 * device, caller order, with respect to the normalized points.  Both walks
 * use Alg. 4's far field whatever wnnc_set_far_field says. */
wnnc_status wnnc_gradient_grad_x(wnnc_ctx ctx, const float *n, const float *sigma, float w,
                                 const float *v, float *dx_out);

/* Far field of the treecode (an extension for precision control; the
 * paper's Alg. 4 is order 0 without wsafe, the default).
 *   order 0: an accepted node contributes its representative term;
 *   order 1, 2: plus the terms of that order of the Taylor expansion of the
 *     pair term about x_B (from the node's moments sum d nu and
 *     sum d d^T nu, d = x - x_B), for nodes of more than one point;
 *   wsafe 1: a node is accepted only if also |x - x_B| > w + sqrt(3) width,
 *     i.e. no point of its cell is within the cutoff w of the target, so
 *     the representative does not carry pairs the cutoff would drop.
 * Applies to every later operator call (winding, gradient, adjoint,
 * queries, orientation).  The moments take 24 floats per node more of
 * device memory while order > 0, and order > 0 takes trees of at most
 * 44,739,242 nodes (2^32 bytes of those moments): WNNC_EINVAL from this
 * call, or from a later build of a larger tree.  Walk plans and tasks are
 * unchanged. */
wnnc_status wnnc_set_far_field(wnnc_ctx ctx, int order, int wsafe);
wnnc_status wnnc_get_far_field(wnnc_ctx ctx, int *order, int *wsafe);

/* Parameter sets of the paper's experiments, for wnnc_orient_preset.  All
 * keep the linear schedule and c = 2, D = 15; widths in the normalized
 * frame. */
#define WNNC_PRESET_DEFAULT 0    /* Sec. 5.1.1: 40 iterations, w1 0.002, w2 0.016 */
#define WNNC_PRESET_NOISE_025 1  /* Sec. 5.2.5, Gaussian noise of 0.25 % of the
                                    bounding-box diagonal: w1 0.02, w2 = 4 w1 */
#define WNNC_PRESET_NOISE_05 2   /* Sec. 5.2.5, 0.5 %: w1 0.03, w2 = 4 w1 */
#define WNNC_PRESET_NOISE_1 3    /* Sec. 5.2.5, 1 %: w1 0.04, w2 = 4 w1 */
#define WNNC_PRESET_SCAN 4       /* Sec. 5.2.6, raw range scans: w1 0.01, w2 0.04 */
#define WNNC_PRESET_HIGH_GENUS 5 /* Sec. 5.2.3, high-genus surfaces: 300
                                    iterations, default widths */

/* Fill *out (host) with preset `preset` (WNNC_PRESET_*): iters, w1, w2 as
 * listed, start_iter 1, stop_iter 0, the linear schedule, no fixed areas.
 * Host only; needs no device. */
wnnc_status wnnc_orient_preset(int preset, wnnc_orient_opts *out);

/* Alg. 3 on the built tree (on every cloud of a batched tree at once, each
 * with its own step length).  mu0: (N,3) initial mu, or NULL for mu = 0 (the
 * paper's initialization).  mu_out: (N,3) final mu (oriented surface
 * elements in the normalized frame; normals are mu_i/|mu_i|).  mu_out may
 * alias mu0.  opts NULL = paper defaults. */
wnnc_status wnnc_orient(wnnc_ctx ctx, const wnnc_orient_opts *opts, const float *mu0,
                        float *mu_out);

/* Output of the method (Alg. 3 result to normals): n_out (N,3) = unit
 * normals mu_i / |mu_i| (zero where mu_i = 0) and, if area_out (N) is not
 * NULL, the solved areas |mu_i| / scale^2 in the frame of the points before
 * wnnc_normalize (scale as returned by it; pass 1 to keep the normalized
 * frame).  mu, n_out, area_out are caller-order device arrays; n_out may
 * alias mu.  Independent of the tree. */
wnnc_status wnnc_normals(wnnc_ctx ctx, const float *mu, int64_t N, double scale, float *n_out,
                         float *area_out);

/* Energies E = ||A_w mu - b||^2 of the mu entering each iteration of the
 * last wnnc_orient, per cloud (host, count * n_clouds doubles; entry
 * k * n_clouds + c is iteration start_iter + k of cloud c; count <= the
 * number of iterations run).  Synchronizes. */
wnnc_status wnnc_orient_energy(wnnc_ctx ctx, double *host_out, int count);

/* Statistics since the last reset (host struct).  Synchronizes. */
wnnc_status wnnc_stats(wnnc_ctx ctx, wnnc_stats_t *out);
wnnc_status wnnc_reset_stats(wnnc_ctx ctx);

/* Copy the octree to host memory for inspection, in the library's node
 * order (depth-first pre-order).  Each array has n_nodes entries except
 * perm (N): depth, leaf flag, and the node's points as the range
 * [begin, end) of the sorted order, whose caller indices are
 * perm[begin..end).  Any pointer may be NULL.  Synchronizes. */
wnnc_status wnnc_tree_export(wnnc_ctx ctx, int32_t *depth, int32_t *leaf, int64_t *begin,
                             int64_t *end, int64_t *perm);

/* nu-representatives for attribute nu in caller order: (N,3) when dim = 3
 * (vector, as for mu) or (N) when dim = 1 (scalar, as for s).  Copies to
 * host, per node in wnnc_tree_export order: x_B (n_nodes,3), nu_B
 * (n_nodes, dim) and the weight W = sum |nu_i| (n_nodes).  Synchronizes. */
wnnc_status wnnc_moments_export(wnnc_ctx ctx, const float *nu, int dim, float *xB, float *nuB,
                                float *W);

/* ------------------------------------------------------- learned warm start
 * A neighbourhood MLP predicts initial normals from the 16 nearest
 * neighbours of each point; the WNNC iteration then starts from them.
 * Network: 48 -> 64 -> 64 -> 3 with ReLU; BF16 operands, FP32 accumulation.
 * Parameters are one device FP32 vector of WNNC_MLP_PARAMS values: W1
 * [48][64], b1 [64], W2 [64][64], b2 [64], W3 [64][3], b3 [3] (row-major
 * [in][out]). */
#define WNNC_MLP_PARAMS 7491

/* Features of every point of the built tree (all clouds), caller order:
 * feat_out (N,48) = offsets to the 16 nearest other points of the same cloud,
 * nearest first (ties by sorted position), divided by their RMS length;
 * rows of clouds with fewer than 17 points are zero-padded.  nbr_out (N,16)
 * int32 caller indices of the neighbours (-1 where missing), or NULL.
 * Points must lie in [-1,1]^3 (normalized). */
wnnc_status wnnc_knn_features(wnnc_ctx ctx, float *feat_out, int32_t *nbr_out);

/* kNN local areas (Sec. 6.1; the estimate Table 5 compares the solved areas
 * with, and a source of fixed areas for wnnc_orient_opts.areas).  For every
 * point of the built tree (all clouds), from its k nearest other points of
 * the same cloud (2 <= k <= 16): the tangent plane of the point and its
 * neighbours by principal components (normal = eigenvector of the smallest
 * eigenvalue of their covariance), the neighbours projected onto it in the
 * basis e1 = the nearest neighbour's projected direction, e2 = n x e1, and
 * the area of the point's Voronoi cell among the projections, clipped to the
 * square [-R,R]^2 (R = the largest projected distance) so that cells at the
 * edge of an open surface stay bounded.  areas_out (N) device, caller order,
 * in the normalized frame (divide by scale^2 for the input frame).  A point
 * with fewer than 2 neighbours gets 0.  FP64 inside, rounded once. */
wnnc_status wnnc_knn_areas(wnnc_ctx ctx, int k, float *areas_out);

/* Unit normals predicted by the MLP: normals_out (N,3) from feat (N,48). */
wnnc_status wnnc_mlp_forward(wnnc_ctx ctx, const float *params, const float *feat, int64_t N,
                             float *normals_out);

/* Loss mean_i (1 - cos(y_i, labels_i)) of the raw MLP outputs y and its
 * gradient with respect to the parameters: grad_out (WNNC_MLP_PARAMS, device).
 * loss_out (host, may be NULL; synchronizes when given). */
wnnc_status wnnc_mlp_grad(wnnc_ctx ctx, const float *params, const float *feat,
                          const float *labels, int64_t N, float *grad_out, double *loss_out);

/* One Adam step (bias-corrected, step >= 1) on params with moments m, v
 * (all WNNC_MLP_PARAMS device floats). */
wnnc_status wnnc_mlp_adam(wnnc_ctx ctx, float *params, float *m, float *v, const float *grad,
                          int step, float lr, float beta1, float beta2, float eps);

/* Warm-started orientation options (defaults in brackets). */
typedef struct {
    int iters;            /* iterations of the warm schedule [6] */
    float w1, w2;         /* warm schedule widths, w2 first [0.002, 0.016]:
                             the plain schedule compressed into `iters` */
    float max_disagree;   /* self-check: largest tolerated fraction of points
                             of a cloud whose final WNNC update points against
                             mu [0.005]; above it the plain method reruns */
    int fallback_iters;   /* plain method iterations on fallback [40] */
    float fallback_w2;    /* plain method initial width on fallback [0.016];
                             its final width is w1 */
    float max_pred_disagree; /* self-check: largest tolerated fraction of
                             points of a cloud whose result points against
                             the prediction [0.4]; near 1/2 the prediction
                             carried no information and the result is
                             not trusted */
    int max_iters;        /* "until convergence" [0: off]: when > iters, the
                             warm schedule is followed by further iterations
                             at width w1, one at a time, while the largest
                             per-cloud fraction of points that the last WNNC
                             update turned against mu (sign changes) exceeds
                             stop_frac and is smaller than after the update
                             before, up to max_iters iterations in all; the
                             self-checks then use the last iteration */
    float stop_frac;      /* sign-change fraction that counts as converged [0] */
} wnnc_warm_opts;

typedef struct {
    int iterations;       /* iterations run (warm + until convergence + fallback) */
    int fallback;         /* 1 if the plain method was rerun */
    double max_disagree;  /* worst per-cloud update self-check fraction */
    double max_pred_disagree; /* worst per-cloud fraction of results against
                             the prediction (before any fallback) */
} wnnc_warm_report;

/* Learned warm start on the built tree (every cloud): neighbourhood
 * features -> MLP unit normals n -> per cloud mu0 = beta n with the
 * least-squares scale beta = <A n, 1/2> / |A n|^2 -> `iters` iterations of
 * Alg. 3 with the warm schedule (then, with max_iters, iterations until the
 * sign changes stop) -> self-checks (the last update and the agreement with
 * the prediction, per cloud); when either fails, the plain method from
 * mu = 0.  mu_out (N,3) as wnnc_orient.  report (host) may be NULL.
 * Synchronizes once (the self-check), and once more per iteration run
 * until convergence. */
wnnc_status wnnc_warm_orient(wnnc_ctx ctx, const float *params, const wnnc_warm_opts *opts,
                             float *mu_out, wnnc_warm_report *report);

/* Message of the last failing call on this thread. */
const char *wnnc_last_error(void);

/* Library version string. */
const char *wnnc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WNNC_H */
