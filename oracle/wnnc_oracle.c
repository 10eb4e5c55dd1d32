/*
 * wnnc_oracle.c -- FP64 CPU oracle for the WNNC operators.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference the GPU
 * library is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load it; the library never does, and this
 * file shares no code, header, table or helper with the GPU path.
 *
 * Everything is double precision.  Point arrays are row-major (n, 3) in the
 * caller's order.  Notation follows the paper (Lin, Shi, Liu 2024,
 * "Fast and Globally Consistent Normal Orientation based on the Winding
 * Number Normal Consistency"):
 *
 *   Phi(y)      = 1 / (4 pi |y|)                       (Thm. 1)
 *   grad Phi(y) = -y / (4 pi |y|^3)                    (Thm. 1)
 *   H Phi(y)    = -I/(4 pi |y|^3) + 3 y y^T/(4 pi |y|^5)  (Sec. 4.2)
 *
 *   A  : mu -> s,     s_i   = sum_j gradPhi(x_i - x_j) . mu_j     (Sec. 4.3, E)
 *   A^T: rho -> v,    v_j   = sum_i rho_i gradPhi(x_i - x_j)      (Alg. 2)
 *   G  : mu -> mu^,   mu^_i = -grad F(x_i; mu)
 *                            = -sum_j HPhi(x_i - x_j) mu_j        (Sec. 4.2)
 *   P  : g -> p,      p_k   = -sum_i g_i HPhi(x_k - x_i) mu_k     (position
 *        gradient of the winding number, an extension: with L = sum_i g_i s_i,
 *        dL/dx_k = -g_k G(mu)_k + p_k; the source attribute is the scalar g,
 *        the target carries its own vector mu_k)
 *   T  : a -> t,      t_k   = sum_j T3Phi(x_k - x_j)[b_k, a_j]       (position
 *        gradient of grad F, an extension: with L = sum_i v_i . grad F(x_i; mu),
 *        dL/dx_k = T(mu; v)_k + T(v; mu)_k; T3Phi is the third derivative
 *        tensor of Phi, the source attribute is the vector a, the target
 *        carries its own vector b)
 *
 * Smoothing (Sec. 4.4): a pair term is set to 0 when |x_i - x_j| < w.  The
 * coincident pair |y| = 0 is also 0 (it is excluded for every w > 0 anyway).
 *
 * Treecode (Sec. 4.5, Alg. 4): an octree over [-1,1]^3 is built by recursive
 * partition; a node is split while it holds more than `leaf_cap` points
 * (1 in the paper) and its depth is below the maximum depth D (15 in the
 * paper).  Child membership: a coordinate equal to the split plane goes to
 * the upper child.  For attribute nu the node representative sits at
 * x_B = sum |nu_i| x_i / sum |nu_j| and carries nu_B = sum nu_i (eqs. for the
 * nu-representatives).  A node whose weight sum |nu| is 0 carries nothing and
 * is skipped.  Per target, starting from the root: if |x - x_B| > c * width(B)
 * the representative stands for the node (with the w cutoff); otherwise an
 * internal node recurses into its children and a leaf sums its points
 * directly (with the w cutoff).  width(B) = 2^(1 - depth(B)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846
#define OR_OP_A 0
#define OR_OP_AT 1
#define OR_OP_G 2
#define OR_OP_P 3
#define OR_OP_T 4

/* ---------------------------------------------------------------- pairs -- */

/* One pair term: target at xt, source (point or representative) at xs with
 * attribute nu (3 values for A and G, 1 value for A^T).  The 1/(4 pi) factor
 * is applied here so that every term is the paper's expression verbatim.
 * Adds the term to out (1 value for A, 3 for A^T and G) and its magnitude to
 * *mag.  A pair closer than w (or coincident) adds nothing. */
static void pair_term(int op, const double *xt, const double *xs, const double *nu,
                      const double *tv, double w, double *out, double *mag)
{
    double y[3] = {xt[0] - xs[0], xt[1] - xs[1], xt[2] - xs[2]};
    double r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    double r = sqrt(r2);
    if (r == 0.0 || r < w)
        return;
    double r3 = r2 * r;
    if (op == OR_OP_A) {
        /* gradPhi(y) . mu = -(y . mu) / (4 pi r^3) */
        double t = -(y[0] * nu[0] + y[1] * nu[1] + y[2] * nu[2]) / (4.0 * OR_PI * r3);
        out[0] += t;
        *mag += fabs(t);
    } else if (op == OR_OP_AT) {
        /* target j, source i: rho_i gradPhi(x_i - x_j) = rho_i (x_j - x_i)/(4 pi r^3),
         * and y = x_j - x_i here. */
        double f = nu[0] / (4.0 * OR_PI * r3);
        double t0 = f * y[0], t1 = f * y[1], t2 = f * y[2];
        out[0] += t0;
        out[1] += t1;
        out[2] += t2;
        *mag += sqrt(t0 * t0 + t1 * t1 + t2 * t2);
    } else if (op == OR_OP_T) {
        /* T3Phi(y)[b, a]_m = (3 r^2 (b_m (y.a) + a_m (y.b) + y_m (a.b))
         *                     - 15 y_m (y.a)(y.b)) / (4 pi r^7) */
        double r7 = r3 * r2 * r2;
        double ya = y[0] * nu[0] + y[1] * nu[1] + y[2] * nu[2];
        double yb = y[0] * tv[0] + y[1] * tv[1] + y[2] * tv[2];
        double ab = nu[0] * tv[0] + nu[1] * tv[1] + nu[2] * tv[2];
        double t[3];
        for (int k = 0; k < 3; ++k)
            t[k] = (3.0 * r2 * (tv[k] * ya + nu[k] * yb + y[k] * ab) - 15.0 * y[k] * ya * yb) /
                   (4.0 * OR_PI * r7);
        out[0] += t[0];
        out[1] += t[1];
        out[2] += t[2];
        *mag += sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    } else if (op == OR_OP_P) {
        /* g (-HPhi(y) v) with the target's vector v */
        double r5 = r3 * r2;
        double yv = y[0] * tv[0] + y[1] * tv[1] + y[2] * tv[2];
        double t[3];
        for (int k = 0; k < 3; ++k)
            t[k] = nu[0] * (tv[k] / (4.0 * OR_PI * r3) - 3.0 * yv * y[k] / (4.0 * OR_PI * r5));
        out[0] += t[0];
        out[1] += t[1];
        out[2] += t[2];
        *mag += sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    } else {
        /* -HPhi(y) mu = mu/(4 pi r^3) - 3 (y . mu) y /(4 pi r^5) */
        double r5 = r3 * r2;
        double ym = y[0] * nu[0] + y[1] * nu[1] + y[2] * nu[2];
        double t[3];
        for (int k = 0; k < 3; ++k)
            t[k] = nu[k] / (4.0 * OR_PI * r3) - 3.0 * ym * y[k] / (4.0 * OR_PI * r5);
        out[0] += t[0];
        out[1] += t[1];
        out[2] += t[2];
        *mag += sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    }
}

static int op_in_dim(int op) { return (op == OR_OP_AT || op == OR_OP_P) ? 1 : 3; }
static int op_out_dim(int op) { return op == OR_OP_A ? 1 : 3; }

/* ---------------------------------------------------------- direct sums -- */

/* Exact O(n_src * n_tgt) sums.  tgt may equal src.  out: (n_tgt, out_dim).
 * mag (optional): per target sum of term magnitudes. */
void or_direct_tv(int op, const double *src, int64_t n_src, const double *nu,
                  const double *tgt, int64_t n_tgt, const double *tv, double w, double *out,
                  double *mag)
{
    int din = op_in_dim(op), dout = op_out_dim(op);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_tgt; ++i) {
        double acc[3] = {0, 0, 0}, m = 0.0;
        for (int64_t j = 0; j < n_src; ++j)
            pair_term(op, tgt + 3 * i, src + 3 * j, nu + din * j, tv ? tv + 3 * i : NULL, w,
                      acc, &m);
        for (int k = 0; k < dout; ++k)
            out[dout * i + k] = acc[k];
        if (mag)
            mag[i] = m;
    }
}

void or_direct(int op, const double *src, int64_t n_src, const double *nu,
               const double *tgt, int64_t n_tgt, double w, double *out, double *mag)
{
    or_direct_tv(op, src, n_src, nu, tgt, n_tgt, NULL, w, out, mag);
}

/* ------------------------------------------------------------- octree -- */

typedef struct {
    int depth;
    int leaf;
    int64_t begin, end;      /* member range in tree->order */
    int nchild;
    int64_t child[8];
    double center[3];
} or_node;

typedef struct {
    int64_t n;
    const double *x;         /* borrowed: (n, 3) */
    double *xc;              /* own copy of the points */
    int64_t *order;          /* point indices grouped by node */
    or_node *nodes;
    int64_t nnodes, cap;
    int max_depth, leaf_cap;
    /* per-call representatives */
    double *rep_x, *rep_nu, *rep_w;
    /* per-call far-field moments about x_B (orders 1 and 2):
     * rep_d[k][l] = sum_j d_jk nu_jl, rep_q[k][n][l] = sum_j d_jk d_jn nu_jl,
     * d_j = x_j - x_B (l runs over 1 or 3 attribute components) */
    double *rep_d, *rep_q;
} or_tree;

static int64_t push_node(or_tree *T)
{
    if (T->nnodes == T->cap) {
        T->cap = T->cap ? 2 * T->cap : 1024;
        T->nodes = (or_node *)realloc(T->nodes, (size_t)T->cap * sizeof(or_node));
    }
    memset(&T->nodes[T->nnodes], 0, sizeof(or_node));
    return T->nnodes++;
}

/* Recursive partition of node `id` (points order[begin:end]).  Children are
 * created for non-empty octants only, in octant order
 * oct = (x >= cx) * 4 + (y >= cy) * 2 + (z >= cz). */
static void split(or_tree *T, int64_t id, int64_t *scratch)
{
    or_node nd = T->nodes[id];
    int64_t cnt = nd.end - nd.begin;
    if (cnt <= T->leaf_cap || nd.depth >= T->max_depth) {
        T->nodes[id].leaf = 1;
        return;
    }
    int64_t bucket_n[8] = {0};
    int8_t *oct = (int8_t *)malloc((size_t)cnt);
    for (int64_t k = 0; k < cnt; ++k) {
        const double *p = T->xc + 3 * T->order[nd.begin + k];
        int o = (p[0] >= nd.center[0]) * 4 + (p[1] >= nd.center[1]) * 2 + (p[2] >= nd.center[2]);
        oct[k] = (int8_t)o;
        bucket_n[o]++;
    }
    int64_t start[8], pos[8];
    int64_t s = nd.begin;
    for (int o = 0; o < 8; ++o) {
        start[o] = s;
        pos[o] = s;
        s += bucket_n[o];
    }
    for (int64_t k = 0; k < cnt; ++k)
        scratch[pos[oct[k]]++] = T->order[nd.begin + k];
    memcpy(T->order + nd.begin, scratch + nd.begin, (size_t)cnt * sizeof(int64_t));
    free(oct);
    double q = ldexp(1.0, -(nd.depth + 1)); /* quarter of width: child half-width */
    T->nodes[id].leaf = 0;
    T->nodes[id].nchild = 0;
    for (int o = 0; o < 8; ++o) {
        if (bucket_n[o] == 0)
            continue;
        int64_t c = push_node(T);
        or_node *ch = &T->nodes[c];
        ch->depth = nd.depth + 1;
        ch->begin = start[o];
        ch->end = start[o] + bucket_n[o];
        ch->center[0] = nd.center[0] + ((o & 4) ? q : -q);
        ch->center[1] = nd.center[1] + ((o & 2) ? q : -q);
        ch->center[2] = nd.center[2] + ((o & 1) ? q : -q);
        or_node *par = &T->nodes[id];
        par->child[par->nchild++] = c;
        split(T, c, scratch);
    }
}

or_tree *or_tree_new(const double *x, int64_t n, int max_depth, int leaf_cap)
{
    if (n <= 0 || max_depth < 0 || leaf_cap < 1)
        return NULL;
    or_tree *T = (or_tree *)calloc(1, sizeof(or_tree));
    T->n = n;
    T->max_depth = max_depth;
    T->leaf_cap = leaf_cap;
    T->xc = (double *)malloc((size_t)n * 3 * sizeof(double));
    memcpy(T->xc, x, (size_t)n * 3 * sizeof(double));
    T->x = T->xc;
    T->order = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        T->order[i] = i;
    int64_t *scratch = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t root = push_node(T);
    T->nodes[root].depth = 0;
    T->nodes[root].begin = 0;
    T->nodes[root].end = n;
    T->nodes[root].center[0] = T->nodes[root].center[1] = T->nodes[root].center[2] = 0.0;
    split(T, root, scratch);
    free(scratch);
    T->rep_x = (double *)malloc((size_t)T->nnodes * 3 * sizeof(double));
    T->rep_nu = (double *)malloc((size_t)T->nnodes * 3 * sizeof(double));
    T->rep_w = (double *)malloc((size_t)T->nnodes * sizeof(double));
    return T;
}

void or_tree_free(or_tree *T)
{
    if (!T)
        return;
    free(T->xc);
    free(T->order);
    free(T->nodes);
    free(T->rep_x);
    free(T->rep_nu);
    free(T->rep_w);
    free(T->rep_d);
    free(T->rep_q);
    free(T);
}

int64_t or_tree_nnodes(const or_tree *T) { return T->nnodes; }

/* Export: per node depth, leaf flag, member range [begin,end) into order[],
 * and order[] itself (n entries). */
void or_tree_export(const or_tree *T, int32_t *depth, int32_t *leaf, int64_t *begin,
                    int64_t *end, int64_t *order)
{
    for (int64_t k = 0; k < T->nnodes; ++k) {
        depth[k] = T->nodes[k].depth;
        leaf[k] = T->nodes[k].leaf;
        begin[k] = T->nodes[k].begin;
        end[k] = T->nodes[k].end;
    }
    memcpy(order, T->order, (size_t)T->n * sizeof(int64_t));
}

/* nu-representatives of every node from its own member points (direct
 * sums, no reuse between levels). dim = 3 (vector nu) or 1 (scalar nu). */
static void compute_reps(or_tree *T, const double *nu, int dim)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < T->nnodes; ++k) {
        const or_node *B = &T->nodes[k];
        double W = 0.0, X[3] = {0, 0, 0}, V[3] = {0, 0, 0};
        for (int64_t m = B->begin; m < B->end; ++m) {
            int64_t i = T->order[m];
            const double *v = nu + dim * i;
            double a = dim == 3 ? sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) : fabs(v[0]);
            W += a;
            for (int c = 0; c < 3; ++c)
                X[c] += a * T->x[3 * i + c];
            for (int c = 0; c < dim; ++c)
                V[c] += v[c];
        }
        T->rep_w[k] = W;
        for (int c = 0; c < 3; ++c) {
            T->rep_x[3 * k + c] = W > 0.0 ? X[c] / W : 0.0;
            T->rep_nu[3 * k + c] = V[c];
        }
    }
}

/* Far-field moments of every node about its x_B (after compute_reps). */
static void compute_moments(or_tree *T, const double *nu, int dim)
{
    if (!T->rep_d) {
        T->rep_d = (double *)malloc((size_t)T->nnodes * 9 * sizeof(double));
        T->rep_q = (double *)malloc((size_t)T->nnodes * 27 * sizeof(double));
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < T->nnodes; ++k) {
        const or_node *B = &T->nodes[k];
        const double *xB = T->rep_x + 3 * k;
        double *D = T->rep_d + 9 * k, *Q = T->rep_q + 27 * k;
        memset(D, 0, 9 * sizeof(double));
        memset(Q, 0, 27 * sizeof(double));
        for (int64_t m = B->begin; m < B->end; ++m) {
            int64_t i = T->order[m];
            const double *v = nu + dim * i;
            double d[3] = {T->x[3 * i] - xB[0], T->x[3 * i + 1] - xB[1], T->x[3 * i + 2] - xB[2]};
            for (int a = 0; a < 3; ++a)
                for (int l = 0; l < dim; ++l)
                    D[3 * a + l] += d[a] * v[l];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    for (int l = 0; l < dim; ++l)
                        Q[9 * a + 3 * b + l] += d[a] * d[b] * v[l];
        }
    }
}

/* Export the representatives of the last call (or compute them for nu). */
void or_tree_reps(or_tree *T, const double *nu, int dim, double *xB, double *nuB, double *W)
{
    compute_reps(T, nu, dim);
    memcpy(xB, T->rep_x, (size_t)T->nnodes * 3 * sizeof(double));
    memcpy(nuB, T->rep_nu, (size_t)T->nnodes * 3 * sizeof(double));
    memcpy(W, T->rep_w, (size_t)T->nnodes * sizeof(double));
}

typedef struct {
    int op;
    double w, c;
    const double *nu;
    int din;
    int order;
    int wsafe; /* also require dist > w + sqrt(3) width (see or_tree_apply_order) */
} apply_args;

/* Derivative tensors of Phi(y) = 1/(4 pi |y|) (the kernel of Thm. 1):
 *   T1_i     = -y_i / (4 pi r^3)
 *   T2_ij    = (3 y_i y_j - r^2 d_ij) / (4 pi r^5)                 (= H Phi)
 *   T3_ijk   = (3 r^2 (d_ij y_k + d_ik y_j + d_jk y_i) - 15 y_i y_j y_k)
 *              / (4 pi r^7)
 *   T4_ijkl  = (105 y_i y_j y_k y_l
 *               - 15 r^2 (d_ij y_k y_l + d_ik y_j y_l + d_il y_j y_k
 *                         + d_jk y_i y_l + d_jl y_i y_k + d_kl y_i y_j)
 *               + 3 r^4 (d_ij d_kl + d_ik d_jl + d_il d_jk)) / (4 pi r^9)
 * each the gradient of the one before. */
static double kd(int i, int j) { return i == j ? 1.0 : 0.0; }

static void phi_derivs(const double *y, double T1[3], double T2[3][3], double T3[3][3][3],
                       double T4[3][3][3][3])
{
    double r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2], r = sqrt(r2);
    double f = 1.0 / (4.0 * OR_PI);
    for (int i = 0; i < 3; ++i) {
        T1[i] = -f * y[i] / (r2 * r);
        for (int j = 0; j < 3; ++j) {
            T2[i][j] = f * (3.0 * y[i] * y[j] - r2 * kd(i, j)) / (r2 * r2 * r);
            for (int k = 0; k < 3; ++k) {
                T3[i][j][k] = f * (3.0 * r2 * (kd(i, j) * y[k] + kd(i, k) * y[j] + kd(j, k) * y[i])
                                   - 15.0 * y[i] * y[j] * y[k]) / (r2 * r2 * r2 * r);
                for (int l = 0; l < 3; ++l)
                    T4[i][j][k][l] =
                        f * (105.0 * y[i] * y[j] * y[k] * y[l]
                             - 15.0 * r2 * (kd(i, j) * y[k] * y[l] + kd(i, k) * y[j] * y[l]
                                            + kd(i, l) * y[j] * y[k] + kd(j, k) * y[i] * y[l]
                                            + kd(j, l) * y[i] * y[k] + kd(k, l) * y[i] * y[j])
                             + 3.0 * r2 * r2 * (kd(i, j) * kd(k, l) + kd(i, k) * kd(j, l)
                                                + kd(i, l) * kd(j, k)))
                        / (r2 * r2 * r2 * r2 * r);
            }
        }
    }
}

/* Far term of node id for target xt, with the Taylor expansion of the pair
 * term about x_B to `order` (0: the representative term of Alg. 4).  With
 * y = xt - x_B and a source at x_B + d, each term f(y - d) is expanded as
 * f(y) - d_k df/dy_k + (1/2) d_k d_n d2f/dy_k dy_n, summed over the node's
 * sources through the moments nu_B, D, Q:
 *   A  : f = T1 . nu         -> T1_l nu_l - T2_lk D_kl + 1/2 T3_lkn Q_knl
 *   A^T: f_m = -rho T1_m     -> -T1_m rho + T2_mk D_k - 1/2 T3_mkn Q_kn
 *   G  : f_m = -T2_ml nu_l   -> -T2_ml nu_l + T3_mlk D_kl - 1/2 T4_mlkn Q_knl
 * (the order-0 parts are the pair terms of pair_term).  Zero, like the
 * order-0 term, when |y| < w or y = 0. */
static void far_term(const or_tree *T, const apply_args *a, int64_t id, const double *xt,
                     const double *tv, double *acc, double *mag)
{
    const double *xB = T->rep_x + 3 * id, *nuB = T->rep_nu + 3 * id;
    if (a->order == 0) {
        pair_term(a->op, xt, xB, nuB, tv, a->w, acc, mag);
        return;
    }
    double y[3] = {xt[0] - xB[0], xt[1] - xB[1], xt[2] - xB[2]};
    double r = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    if (r == 0.0 || r < a->w)
        return;
    double T1[3], T2[3][3], T3[3][3][3], T4[3][3][3][3];
    phi_derivs(y, T1, T2, T3, T4);
    const double *D = T->rep_d + 9 * id, *Q = T->rep_q + 27 * id;
    const double o2 = a->order >= 2 ? 1.0 : 0.0;
    double t[3] = {0, 0, 0};
    if (a->op == OR_OP_A) {
        for (int l = 0; l < 3; ++l) {
            t[0] += T1[l] * nuB[l];
            for (int k = 0; k < 3; ++k) {
                t[0] -= T2[l][k] * D[3 * k + l];
                for (int n = 0; n < 3; ++n)
                    t[0] += o2 * 0.5 * T3[l][k][n] * Q[9 * k + 3 * n + l];
            }
        }
        acc[0] += t[0];
        *mag += fabs(t[0]);
        return;
    }
    for (int m = 0; m < 3; ++m) {
        if (a->op == OR_OP_AT) {
            t[m] -= T1[m] * nuB[0];
            for (int k = 0; k < 3; ++k) {
                t[m] += T2[m][k] * D[3 * k];
                for (int n = 0; n < 3; ++n)
                    t[m] -= o2 * 0.5 * T3[m][k][n] * Q[9 * k + 3 * n];
            }
        } else {
            for (int l = 0; l < 3; ++l) {
                t[m] -= T2[m][l] * nuB[l];
                for (int k = 0; k < 3; ++k) {
                    t[m] += T3[m][l][k] * D[3 * k + l];
                    for (int n = 0; n < 3; ++n)
                        t[m] -= o2 * 0.5 * T4[m][l][k][n] * Q[9 * k + 3 * n + l];
                }
            }
        }
    }
    for (int m = 0; m < 3; ++m)
        acc[m] += t[m];
    *mag += sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
}

/* Decision margins of one target (diagnostics; they change no result):
 * mg[0] = the smallest |dist - thr| / thr over the acceptance tests the
 * target evaluated (thr the distance Alg. 4 compares with), mg[1] = the
 * smallest |r - w| / w over the pair terms it formed, representatives and
 * points alike (the cutoff of Sec. 4.4; only for w > 0).  A decision whose
 * margin is far below one is one that a few roundings of the distance can
 * turn. */
static void note_margin(double *mg, int k, double r, double thr)
{
    if (mg && thr > 0.0) {
        double m = fabs(r - thr) / thr;
        if (m < mg[k])
            mg[k] = m;
    }
}

/* Alg. 4 for one target xt (with its vector tv for P) starting at node id;
 * mg (NULL or 2 doubles) collects the decision margins. */
static void apply_node(const or_tree *T, const apply_args *a, int64_t id, const double *xt,
                       const double *tv, double *acc, double *mag, int64_t *pairs, double *mg)
{
    const or_node *B = &T->nodes[id];
    if (T->rep_w[id] == 0.0)
        return; /* nothing to carry: every attribute in B is zero */
    const double *xB = T->rep_x + 3 * id;
    double dx = xt[0] - xB[0], dy = xt[1] - xB[1], dz = xt[2] - xB[2];
    double dist = sqrt(dx * dx + dy * dy + dz * dz);
    double width = ldexp(2.0, -B->depth);
    double thr = a->c * width;
    if (a->wsafe && a->w + sqrt(3.0) * width > thr)
        thr = a->w + sqrt(3.0) * width;
    note_margin(mg, 0, dist, thr);
    if (dist > thr) {
        note_margin(mg, 1, dist, a->w);
        far_term(T, a, id, xt, tv, acc, mag);
        (*pairs)++;
    } else if (!B->leaf) {
        for (int k = 0; k < B->nchild; ++k)
            apply_node(T, a, B->child[k], xt, tv, acc, mag, pairs, mg);
    } else {
        for (int64_t m = B->begin; m < B->end; ++m) {
            int64_t j = T->order[m];
            const double *xj = T->x + 3 * j;
            if (mg) {
                double ex = xt[0] - xj[0], ey = xt[1] - xj[1], ez = xt[2] - xj[2];
                note_margin(mg, 1, sqrt(ex * ex + ey * ey + ez * ez), a->w);
            }
            pair_term(a->op, xt, xj, a->nu + a->din * j, tv, a->w, acc, mag);
            (*pairs)++;
        }
    }
}

/* Treecode operator over targets tgt (n_tgt x 3).  Computes the
 * representatives for nu first (every call, as they move with nu).
 * out: (n_tgt, out_dim); mag, pairs optional per-target outputs.
 *
 * Extensions (not in the paper; precision control): `order` 1 or 2 uses
 * the Taylor expansion of the pair term about x_B for accepted nodes
 * (far_term); `wsafe` accepts a node only if, besides Alg. 4's test, the
 * target is farther than w + sqrt(3) width from x_B: x_B lies in the
 * node's cell, whose points are all within sqrt(3) width of it, so no
 * accepted node holds a point the cutoff w would drop.
 * margins (optional, (n_tgt, 2)): per target the decision margins of
 * note_margin. */
void or_tree_apply_margins(or_tree *T, int op, const double *nu, double w, double c, int order,
                           int wsafe, const double *tgt, int64_t n_tgt, const double *tv,
                           double *out, double *mag, int64_t *pairs, double *margins)
{
    int din = op_in_dim(op), dout = op_out_dim(op);
    if (op == OR_OP_P || op == OR_OP_T)
        order = 0; /* P, T: the representative term only */
    compute_reps(T, nu, din);
    if (order > 0)
        compute_moments(T, nu, din);
    apply_args a = {op, w, c, nu, din, order, wsafe};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_tgt; ++i) {
        double acc[3] = {0, 0, 0}, m = 0.0;
        int64_t np = 0;
        double *mg = margins ? margins + 2 * i : NULL;
        if (mg)
            mg[0] = mg[1] = HUGE_VAL;
        apply_node(T, &a, 0, tgt + 3 * i, tv ? tv + 3 * i : NULL, acc, &m, &np, mg);
        for (int k = 0; k < dout; ++k)
            out[dout * i + k] = acc[k];
        if (mag)
            mag[i] = m;
        if (pairs)
            pairs[i] = np;
    }
}

/* Treecode operator without the decision margins. */
void or_tree_apply_tv(or_tree *T, int op, const double *nu, double w, double c, int order,
                      int wsafe, const double *tgt, int64_t n_tgt, const double *tv,
                      double *out, double *mag, int64_t *pairs)
{
    or_tree_apply_margins(T, op, nu, w, c, order, wsafe, tgt, n_tgt, tv, out, mag, pairs, NULL);
}

void or_tree_apply_order(or_tree *T, int op, const double *nu, double w, double c, int order,
                         int wsafe, const double *tgt, int64_t n_tgt, double *out, double *mag,
                         int64_t *pairs)
{
    or_tree_apply_tv(T, op, nu, w, c, order, wsafe, tgt, n_tgt, NULL, out, mag, pairs);
}

void or_tree_apply(or_tree *T, int op, const double *nu, double w, double c,
                   const double *tgt, int64_t n_tgt, double *out, double *mag, int64_t *pairs)
{
    or_tree_apply_order(T, op, nu, w, c, 0, 0, tgt, n_tgt, out, mag, pairs);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
