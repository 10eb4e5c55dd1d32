"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formula: each compares it with a closed
form, an identity that needs different arithmetic, a hand-computed value, a
special case, brute force on a tiny input, or a number printed in the paper.
"""
import numpy as np
import pytest

import synth

FOUR_PI = 4.0 * np.pi


def exact_sphere(n):
    s = synth.fibonacci_sphere(n, seed=0, jitter=0.0, with_init=False)
    x = s.points.astype(np.float64)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x


# ------------------------------------------------------- Sec. 5.1.1 input --

def test_normalize_by_hand(oracle_mod):
    """Sec. 5.1.1 reading: centre = midpoint of the bounding box, one uniform
    scale so that the largest half-extent is 10/11.  Points (0,0,0) and
    (2,4,6): centre (1,2,3), largest half-extent 3, scale (10/11)/3, and the
    extreme z coordinates become -10/11 and +10/11."""
    p = np.array([[0.0, 0.0, 0.0], [2.0, 4.0, 6.0]], np.float32)
    x, centre, scale = oracle_mod.normalize(p)
    assert np.array_equal(centre, [1.0, 2.0, 3.0])
    assert scale == pytest.approx((10.0 / 11.0) / 3.0, rel=1e-15)
    assert x.dtype == np.float32
    assert x[0, 2] == np.float32(-10.0 / 11.0) and x[1, 2] == np.float32(10.0 / 11.0)
    # uniform scale: the aspect ratio 1:2:3 is kept
    assert np.array_equal(x[1], np.float32([10.0 / 33.0, 20.0 / 33.0, 10.0 / 11.0]))


def test_normalize_centre_is_the_box_midpoint_not_the_mean(oracle_mod):
    """An off-centre cloud (mean != midpoint): four points at x = 0 and one
    at x = 10 (mean 2, midpoint 5); the extremes map to -10/11 and 10/11,
    and y, z (extent 1) keep the scale of x (1/11 per unit)."""
    p = np.array([[0, 0, 0], [0, 1, 0], [0, 0, 1], [0, 1, 1], [10, 0.5, 0.5]], np.float32)
    x, centre, scale = oracle_mod.normalize(p)
    assert centre[0] == 5.0 and centre[1] == 0.5 and centre[2] == 0.5
    assert scale == pytest.approx(2.0 / 11.0, rel=1e-15)
    assert x[0, 0] == np.float32(-10.0 / 11.0) and x[4, 0] == np.float32(10.0 / 11.0)
    assert x[1, 1] == np.float32(1.0 / 11.0) and x[0, 1] == np.float32(-1.0 / 11.0)
    assert np.abs(x).max() == np.float32(10.0 / 11.0)


def test_normalize_is_invariant_to_exact_affine_changes(oracle_mod):
    """Translating by a dyadic vector and scaling by a power of two change
    neither the FP32 result (every step is exact), and the largest
    half-extent always lands on 10/11."""
    rng = np.random.default_rng(5)
    # coordinates on a grid of 1/1024 with at most 14 significant bits, so
    # the change below and the normalization's differences are exact
    p = (rng.integers(-3000, 7000, size=(500, 3)) / 1024.0).astype(np.float32)
    x0, c0, s0 = oracle_mod.normalize(p)
    t = np.array([0.5, -2.25, 16.0])
    q = (p.astype(np.float64) * 8.0 + t).astype(np.float32)
    assert np.array_equal((q.astype(np.float64) - t) / 8.0, p)
    x1, c1, s1 = oracle_mod.normalize(q)
    assert np.array_equal(c1, 8.0 * c0 + t) and s1 == s0 / 8.0
    assert np.array_equal(x1, x0)
    half = (x0.max(0).astype(np.float64) - x0.min(0)) / 2
    assert half.max() == pytest.approx(10.0 / 11.0, rel=1e-7)


# ----------------------------------------------------------------- Thm. 1 --

@pytest.mark.parametrize("n", [500, 2000])
def test_sphere_centre_is_exactly_one(oracle_mod, n):
    """Thm. 1 / eq. (wnf-discretization): with x_j on the unit sphere,
    mu_j = sigma x_j and sigma = 4 pi / N, every term at the centre equals
    sigma / (4 pi), so F(0) = 1 exactly for any N."""
    x = exact_sphere(n)
    mu = x * (FOUR_PI / n)
    q = np.zeros((1, 3))
    for f in (oracle_mod.direct("A", x, mu, 1e-3, targets=q),
              oracle_mod.direct_np.A(x, mu, 1e-3, targets=q),
              # the same sphere shrunk to radius 0.9 (inside the root cube),
              # with the area weights scaled by 0.9^2
              oracle_mod.Tree(x * 0.9).apply("A", mu * 0.81, 1e-3, c=1e9, targets=q)):
        assert abs(float(f[0]) - 1.0) < 1e-12


def test_inside_outside_indicator(oracle_mod):
    """Thm. 1: F is 1 inside, 0 outside (quadrature error of a 2000-point
    Fibonacci rule away from the surface is small)."""
    x = exact_sphere(2000)
    mu = x * (FOUR_PI / 2000)
    inside = np.array([[0.3, -0.2, 0.1], [0.0, 0.5, -0.4], [-0.6, 0.0, 0.0]])
    outside = np.array([[3.0, 0.2, 0.1], [0.0, -1.6, 0.0], [1.0, 1.0, 1.0]])
    fi = oracle_mod.direct("A", x, mu, 1e-3, targets=inside)
    fo = oracle_mod.direct("A", x, mu, 1e-3, targets=outside)
    assert np.all(np.abs(fi - 1.0) < 2e-3)
    assert np.all(np.abs(fo) < 2e-3)


def test_on_surface_coulomb_identity(oracle_mod):
    """On the unit sphere (x_j - x_i) . x_j = r_ij^2 / 2, so with mu_j = sigma
    x_j the discretized winding number at x_i equals the Coulomb sum
    (sigma / 8 pi) sum_{j != i} 1/r_ij -- a different formula evaluated with
    different arithmetic.  Its continuum value is 1/2 (Thm. 1 on the
    boundary); the excluded self cell biases it down by about
    sqrt(sigma/pi)/4."""
    n = 2000
    x = exact_sphere(n)
    sigma = FOUR_PI / n
    s = oracle_mod.direct("A", x, x * sigma, 1e-4)
    r = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(axis=2))
    np.fill_diagonal(r, np.inf)
    coul = sigma / (8 * np.pi) * (1.0 / r).sum(axis=1)
    assert np.max(np.abs(s - coul)) < 1e-12
    bias = np.sqrt(sigma / np.pi) / 4
    assert abs(s.mean() - (0.5 - bias)) < 2e-3


def test_sphere_normals_are_a_wnnc_fixed_point(oracle_mod):
    """Sec. 4.2, eq. (wnnc-property-v2): outward sphere normals satisfy
    mu_i = lambda_i G(mu)_i with lambda_i > 0.  On the unit sphere with
    mu_j = sigma x_j the gradient operator reduces to the closed form
    G_i = (sigma/4pi) sum_{j != i} [(3/2) x_i - (1/2) x_j] / r_ij^3."""
    n = 2000
    x = exact_sphere(n)
    sigma = FOUR_PI / n
    g = oracle_mod.direct("G", x, x * sigma, 1e-4)
    gnp = oracle_mod.direct_np.G(x, x * sigma, 1e-4)
    d = x[:, None, :] - x[None, :, :]
    r = np.sqrt((d ** 2).sum(axis=2))
    np.fill_diagonal(r, np.inf)
    closed = sigma / FOUR_PI * ((1.5 * x[:, None, :] - 0.5 * x[None, :, :]) / r[:, :, None] ** 3).sum(axis=1)
    assert np.max(np.abs(g - closed)) / np.max(np.abs(closed)) < 1e-11
    assert np.max(np.abs(gnp - closed)) / np.max(np.abs(closed)) < 1e-11
    cosang = (g * x).sum(1) / np.linalg.norm(g, axis=1)
    assert np.all(cosang > 0.999)


# ------------------------------------------------------ hand computations --

def test_two_point_hand_values(oracle_mod):
    """x1 = 0, x2 = (1/2,0,0), mu2 = (1,0,0), r = 1/2, 4 pi r^3 = pi/2,
    4 pi r^5 = pi/8:
      A at x1      = -(x1-x2).mu2 / (pi/2)                  = 1/pi
      G at x1      = mu2/(pi/2) - 3 (y.mu2) y/(pi/8)        = (-4/pi, 0, 0)
      A^T(rho=(1,0)) at x2 = rho1 (x2-x1)/(pi/2)            = (1/pi, 0, 0)."""
    x = np.array([[0.0, 0, 0], [0.5, 0, 0]])
    mu = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    for mod in ("c", "np"):
        A = oracle_mod.direct("A", x, mu, 0.1) if mod == "c" else oracle_mod.direct_np.A(x, mu, 0.1)
        G = oracle_mod.direct("G", x, mu, 0.1) if mod == "c" else oracle_mod.direct_np.G(x, mu, 0.1)
        rho = np.array([1.0, 0.0])
        AT = oracle_mod.direct("AT", x, rho, 0.1) if mod == "c" else oracle_mod.direct_np.AT(x, rho, 0.1)
        assert np.allclose(A, [1 / np.pi, 0.0], rtol=0, atol=1e-15)
        assert np.allclose(G[0], [-4 / np.pi, 0, 0], rtol=0, atol=1e-14)
        assert np.allclose(G[1], [0, 0, 0], atol=1e-15)
        assert np.allclose(AT[1], [1 / np.pi, 0, 0], rtol=0, atol=1e-15)
        assert np.allclose(AT[0], [0, 0, 0], atol=1e-15)
    # the smoothing width removes the pair (Sec. 4.4: zero when |y| < w)
    assert np.all(oracle_mod.direct("A", x, mu, 0.5000001) == 0.0)
    assert np.any(oracle_mod.direct("A", x, mu, 0.5) != 0.0)


def test_gradient_is_minus_grad_of_winding_number(oracle_mod):
    """G(mu)_i = -grad F(x_i; mu) (Sec. 4.2): central differences of the
    winding number queried off the points; the self term stays cut off on
    both sides since h < w."""
    rng = np.random.default_rng(11)
    x = rng.uniform(-0.8, 0.8, size=(40, 3))
    mu = rng.standard_normal((40, 3)) * 0.01
    w, h = 1e-3, 1e-6
    g = oracle_mod.direct("G", x, mu, w)
    for i in range(0, 40, 7):
        fd = np.zeros(3)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            fp = oracle_mod.direct("A", x, mu, w, targets=(x[i] + e)[None])
            fm = oracle_mod.direct("A", x, mu, w, targets=(x[i] - e)[None])
            fd[k] = -(fp[0] - fm[0]) / (2 * h)
        assert np.allclose(fd, g[i], rtol=1e-6, atol=1e-8 * np.abs(g[i]).max())


def test_adjoint_and_symmetry(oracle_mod):
    """<A mu, s> = <mu, A^T s> and <G u, v> = <u, G v> for the exact sums
    (gradPhi is odd and HPhi is even and symmetric)."""
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, size=(300, 3))
    mu, u, v = (rng.standard_normal((300, 3)) for _ in range(3))
    s = rng.standard_normal(300)
    for w in (0.0, 0.05):
        lhs = float(oracle_mod.direct("A", x, mu, w) @ s)
        rhs = float((mu * oracle_mod.direct("AT", x, s, w)).sum())
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
        gl = float((oracle_mod.direct("G", x, u, w) * v).sum())
        gr = float((u * oracle_mod.direct("G", x, v, w)).sum())
        assert abs(gl - gr) <= 1e-12 * max(abs(gl), 1.0)


# ---------------------------------------------------------------- Alg. 2 --

def test_grad_step_is_an_exact_line_search(oracle_mod):
    """Alg. 2 minimises ||A mu - b||^2 along r exactly: the new gradient
    A^T(A mu' - b) is orthogonal to r, and the energy does not increase."""
    from oracle.iterate import _Ops, grad_step
    rng = np.random.default_rng(5)
    x = rng.uniform(-0.9, 0.9, size=(200, 3))
    ops = _Ops(x, "direct")
    mu = rng.standard_normal((200, 3)) * 1e-3
    mu1, alpha, r, E0 = grad_step(ops, mu, 0.01)
    g1 = ops("AT", ops("A", mu1, 0.01) - 0.5, 0.01)
    assert abs(float((g1 * r).sum())) < 1e-9 * float((r * r).sum())
    E1 = float(((ops("A", mu1, 0.01) - 0.5) ** 2).sum())
    assert alpha > 0 and E1 < E0


# -------------------------------------------------------------- treecode --

def tree_sets(T):
    depth, leaf, begin, end, order = T.export()
    return {(int(d), tuple(sorted(order[b:e]))) for d, b, e in zip(depth, begin, end)}, depth, leaf, begin, end, order


def test_tree_hand_cases(oracle_mod):
    """Sec. 4.5: partition until one point or depth D; the cube is [-1,1]^3."""
    # opposite octants: root + two depth-1 leaves
    T = oracle_mod.Tree(np.array([[-0.5, -0.5, -0.5], [0.5, 0.5, 0.5]]))
    sets = tree_sets(T)[0]
    assert sets == {(0, (0, 1)), (1, (0,)), (1, (1,))}
    # 0.1 and 0.2 share the cells [0,1], [0,.5], [0,.25] and split at 0.125
    T = oracle_mod.Tree(np.array([[0.1, 0.1, 0.1], [0.2, 0.1, 0.1]]))
    sets = tree_sets(T)[0]
    assert sets == {(0, (0, 1)), (1, (0, 1)), (2, (0, 1)), (3, (0, 1)), (4, (0,)), (4, (1,))}
    # coincident points: a chain to the depth limit, one leaf holding all
    T = oracle_mod.Tree(np.array([[0.3, -0.2, 0.7]] * 3), max_depth=15)
    sets, depth, leaf, begin, end, _ = tree_sets(T)
    assert len(sets) == 16 and (15, (0, 1, 2)) in sets
    assert leaf[depth == 15].all() and not leaf[depth < 15].any()
    # a coordinate on the split plane goes to the upper child
    T = oracle_mod.Tree(np.array([[0.0, 0.0, 0.0], [-1e-12, 0.0, 0.0]]))
    sets = tree_sets(T)[0]
    assert sets == {(0, (0, 1)), (1, (0,)), (1, (1,))}
    # a shallower maximum depth stops the chain
    T = oracle_mod.Tree(np.array([[0.3, -0.2, 0.7]] * 2), max_depth=4)
    assert T.nnodes == 5


def test_tree_invariants(oracle_mod):
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.uniform(-1, 1, (3000, 3)), np.repeat(rng.uniform(-1, 1, (5, 3)), 4, axis=0)])
    T = oracle_mod.Tree(x)
    depth, leaf, begin, end, order = T.export()
    assert sorted(order.tolist()) == list(range(len(x)))
    cnt = end - begin
    # leaf iff one point or maximum depth; every point in exactly one leaf
    assert np.all((cnt[leaf == 1] == 1) | (depth[leaf == 1] == 15))
    assert np.all(cnt[leaf == 0] > 1)
    assert cnt[leaf == 1].sum() == len(x)
    # members of a node lie in its cube: cell index at that depth agrees
    for k in rng.choice(T.nnodes, 200, replace=False):
        pts = x[order[begin[k]:end[k]]]
        cell = np.floor((pts + 1.0) * 2.0 ** (depth[k] - 1))
        cell = np.minimum(cell, 2 ** depth[k] - 1)
        assert np.all(cell == cell[0])


def test_treecode_special_cases(oracle_mod):
    """(i) never accepting (c -> inf) gives the exact sum; (ii) always
    accepting at the root (c -> 0) gives the single monopole term
    gradPhi(x_i - x_B) . nu_B with x_B the |mu|-weighted centroid;
    (iii) positive and negative homogeneity in nu."""
    rng = np.random.default_rng(21)
    x = rng.uniform(-0.9, 0.9, size=(500, 3))
    mu = rng.standard_normal((500, 3)) * 1e-3
    rho = rng.standard_normal(500)
    T = oracle_mod.Tree(x)
    w = 0.01
    for op, nu in (("A", mu), ("AT", rho), ("G", mu)):
        ex = oracle_mod.direct(op, x, nu, w)
        tr = T.apply(op, nu, w, c=1e9)
        assert np.max(np.abs(tr - ex)) <= 1e-12 * np.max(np.abs(ex))
        for lam in (3.0, -2.5):
            ref = lam * T.apply(op, nu, w)
            assert np.max(np.abs(T.apply(op, lam * nu, w) - ref)) <= 1e-12 * np.max(np.abs(ref))
    a = np.linalg.norm(mu, axis=1)
    xB = (a[:, None] * x).sum(0) / a.sum()
    y = x - xB
    r = np.linalg.norm(y, axis=1)
    mono = -(y @ mu.sum(0)) / (FOUR_PI * r ** 3)
    tr = T.apply("A", mu, w, c=1e-9)
    assert np.allclose(tr, mono, rtol=1e-12, atol=0)


def test_accept_test_is_strict_at_a_tie(oracle_mod):
    """Alg. 4 accepts a node only if the target is farther than c 2^(1-d)
    from x_B: at exactly that distance the node is opened.  Two equal-weight
    points share one depth-3 cell (width 1/4) and split at depth 4; x_B is
    their midpoint; a query on the x axis at distance exactly 2 * 1/4 from it
    (every coordinate dyadic, so every distance is exact) opens the node and
    sums both points; a query one ulp farther takes the representative."""
    x = np.array([[0.0625, 0.0625, 0.0625], [0.1875, 0.0625, 0.0625]])
    mu = np.array([[0.01, 0.0, 0.0], [0.01, 0.0, 0.0]])
    T = oracle_mod.Tree(x)
    xb = np.array([0.125, 0.0625, 0.0625])
    tie = xb + np.array([0.5, 0.0, 0.0])
    far = tie.copy()
    far[0] = np.nextafter(far[0], 1.0)
    Q = np.stack([tie, far])
    out, _, pairs = T.apply("A", mu, 1e-3, c=2.0, targets=Q, with_stats=True)
    assert list(pairs) == [2, 1]
    exact = oracle_mod.direct("A", x, mu, 1e-3, targets=Q)
    assert out[0] == pytest.approx(exact[0], rel=1e-14)
    d = far - xb
    mono = -(d @ mu.sum(0)) / (FOUR_PI * np.linalg.norm(d) ** 3)
    assert out[1] == pytest.approx(mono, rel=1e-14)
    assert out[0] != pytest.approx(out[1], rel=1e-6)


def test_decision_margins_by_hand(oracle_mod):
    """The decision margins the oracle reports per target (diagnostics for
    the parity bar): at the acceptance tie above the smallest relative
    margin |dist - c width| / (c width) is exactly 0, one ulp farther it is
    that ulp over c width = 1/2; two points exactly w apart (dyadic, so the
    distance is exact) sit on the cutoff of Sec. 4.4: margin 0, and the pair
    is kept (only |y| < w is dropped)."""
    x = np.array([[0.0625, 0.0625, 0.0625], [0.1875, 0.0625, 0.0625]])
    mu = np.array([[0.01, 0.0, 0.0], [0.01, 0.0, 0.0]])
    T = oracle_mod.Tree(x)
    tie = np.array([0.625, 0.0625, 0.0625])
    far = tie.copy()
    far[0] = np.nextafter(far[0], 1.0)
    out, mg = T.apply("A", mu, 1e-3, c=2.0, targets=np.stack([tie, far]), with_margins=True)
    assert mg[0, 0] == 0.0
    assert mg[1, 0] == (far[0] - tie[0]) / 0.5
    # the results do not depend on the diagnostics
    assert np.array_equal(out, T.apply("A", mu, 1e-3, c=2.0, targets=np.stack([tie, far])))
    y = np.array([[0.0, 0.0, 0.0], [0.125, 0.0, 0.0]])
    m2 = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    T2 = oracle_mod.Tree(y)
    s, mg2 = T2.apply("A", m2, 0.125, c=2.0, with_margins=True)
    assert mg2[0, 1] == 0.0
    assert s[0] == pytest.approx(-(-0.125) / (FOUR_PI * 0.125 ** 3), rel=1e-15)
    # w = 0: no cutoff, no cutoff margin
    _, mg3 = T2.apply("A", m2, 0.0, c=2.0, with_margins=True)
    assert np.all(np.isinf(mg3[:, 1]))


def test_treecode_zero_weight_nodes_are_skipped(oracle_mod):
    """A node whose attributes are all zero carries no representative; a
    zero input gives exactly zero with no pair evaluated."""
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, size=(400, 3))
    T = oracle_mod.Tree(x)
    out, mag, pairs = T.apply("A", np.zeros((400, 3)), 0.01, with_stats=True)
    assert np.all(out == 0) and np.all(pairs == 0)


def test_treecode_error_shrinks_with_c(oracle_mod):
    """The far-field approximation error decreases as the acceptance
    threshold c grows (c = 2 is the paper's setting)."""
    cl = synth.ellipsoid_union(6000, seed=4, noise=0.0, with_init=False)
    x, _, sc = oracle_mod.normalize(cl.points)
    x = x.astype(np.float64)
    mu = cl.normals.astype(np.float64) * (cl.area * sc * sc / len(x))
    ex = oracle_mod.direct("G", x, mu, 0.002)
    T = oracle_mod.Tree(x)
    errs = [np.linalg.norm(T.apply("G", mu, 0.002, c=c) - ex) / np.linalg.norm(ex) for c in (1.0, 2.0, 4.0)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 2e-2


# ---------------------------------------------------------------- Alg. 3 --

def test_iteration_ablations(oracle_mod):
    """Sec. 5.5.2: without the gradient step mu stays exactly 0; without the
    rescale one WNNC update changes the lengths by a large factor that grows
    with the point density (10^4..10^10 on the paper's data)."""
    factors = []
    for n in (800, 3200):
        s = synth.fibonacci_sphere(n, 0, with_init=False)
        x, _, _ = oracle_mod.normalize(s.points)
        if n == 800:
            mu = oracle_mod.orient(x, iters=5, backend="direct", grad=False)
            assert np.all(mu == 0)
        seen, ref = [], []
        oracle_mod.orient(x, iters=1, backend="direct", do_rescale=False,
                          callback=lambda i, m, info: seen.append(np.linalg.norm(m, axis=1).mean()))
        oracle_mod.orient(x, iters=1, backend="direct",
                          callback=lambda i, m, info: ref.append(np.linalg.norm(m, axis=1).mean()))
        factors.append(seen[0] / ref[0])
    assert factors[0] > 100 and factors[1] > 4 * factors[0]


def test_flipping_mu_flips_every_operator(oracle_mod):
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, size=(200, 3))
    mu = rng.standard_normal((200, 3))
    for op in ("A", "G"):
        assert np.array_equal(oracle_mod.direct(op, x, -mu, 0.01), -oracle_mod.direct(op, x, mu, 0.01))


def test_sphere_end_to_end_direct(oracle_mod):
    """Alg. 3 from mu = 0 on the 2k jittered sphere orients every normal
    outward (Sec. 4.3: zero initialisation and the PGR energy resolve the
    inside/outside ambiguity)."""
    s = synth.fibonacci_sphere(2000, 0)
    x, _, sc = oracle_mod.normalize(s.points)
    mu = oracle_mod.orient(x, backend="direct")
    n = mu / np.linalg.norm(mu, axis=1, keepdims=True)
    dots = (n * s.normals).sum(1)
    assert np.all(dots > 0)
    assert ((1 - dots) / 2).mean() < 2e-4
    # unscaled unit random initial vectors break it (Sec. 6.1.3)
    mu_r = oracle_mod.orient(x, backend="direct", iters=10, mu0=s.mu0.astype(np.float64))
    assert ((mu_r * s.normals).sum(1) > 0).mean() < 0.9


@pytest.mark.slow
def test_table5_sphere_areas(oracle_mod):
    """Table 5: 40 iterations of the treecode method on the 163,842-vertex
    unit sphere; total and mean solved area agree with the printed values
    (the frame is the unit sphere: the normalized areas are divided by the
    square of the normalization scale)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table5_sphere_areas.txt")
    rows = {}
    for line in open(path):
        if line.startswith("#") or line.startswith("stat") or not line.strip():
            continue
        k, gt, knn, solved = line.split()
        rows[k] = float(solved)
    s = synth.icosphere(7)
    assert s.n == 163842
    x, _, sc = oracle_mod.normalize(s.points)
    mu = oracle_mod.orient(x, backend="tree")
    a = np.linalg.norm(mu, axis=1) / sc ** 2
    assert abs(a.sum() / rows["total"] - 1) < 1e-3
    assert abs(a.mean() / rows["mean"] - 1) < 1e-3
    # the extremes are looser: the paper's sphere triangulation is not
    # specified beyond its vertex count
    assert abs(a.min() / rows["min"] - 1) < 0.05
    assert abs(a.max() / rows["max"] - 1) < 0.05
    n = mu / np.linalg.norm(mu, axis=1, keepdims=True)
    assert np.all((n * s.normals).sum(1) > 0)


# ------------------------------- method variants (Sec. 5.5.1, Sec. 6.1.1)

def test_width_schedules_end_points_and_shape(oracle_mod):
    """Every schedule starts at w2, ends at w1 and decreases; the cosine
    midpoint is the mean and the exponential midpoint the geometric mean;
    the linear one is Alg. 3's formula."""
    from oracle.iterate import width_schedule
    w1, w2 = 0.002, 0.016
    for mode in ("linear", "cosine", "exponential"):
        ws = [width_schedule(i, 41, w1, w2, mode) for i in range(1, 42)]
        assert ws[0] == pytest.approx(w2, rel=1e-15)
        assert ws[-1] == pytest.approx(w1, rel=1e-15)
        assert all(a >= b for a, b in zip(ws, ws[1:]))
        assert width_schedule(1, 1, w1, w2, mode) == w1
    assert width_schedule(21, 41, w1, w2, "cosine") == pytest.approx((w1 + w2) / 2, rel=1e-14)
    assert width_schedule(21, 41, w1, w2, "exponential") == pytest.approx(np.sqrt(w1 * w2), rel=1e-14)
    assert width_schedule(11, 41, w1, w2, "linear") == pytest.approx(w2 - 0.25 * (w2 - w1), rel=1e-14)
    with pytest.raises(ValueError):
        width_schedule(2, 5, 0.0, w2, "exponential")


def test_fixed_area_rescale_sets_the_lengths(oracle_mod):
    """Sec. 6.1.1: |mu_i| = sigma_i with the direction of G(mu)_i; a zero
    G keeps mu_i.  On the sphere with sigma = 4 pi / N the run orients every
    point outward and ends with exactly those lengths."""
    from oracle import iterate
    rng = np.random.default_rng(4)
    mu = rng.standard_normal((6, 3))
    g = rng.standard_normal((6, 3))
    g[2] = 0.0
    sig = rng.uniform(0.5, 2.0, 6)
    out = iterate.rescale(mu, g, sig)
    ok = np.arange(6) != 2
    assert np.allclose(np.linalg.norm(out[ok], axis=1), sig[ok], rtol=1e-14)
    assert np.allclose(out[ok] / np.linalg.norm(out[ok], axis=1)[:, None],
                       g[ok] / np.linalg.norm(g[ok], axis=1)[:, None], rtol=1e-14)
    assert np.array_equal(out[2], mu[2])
    c = synth.fibonacci_sphere(2000, 0)
    x, _, _ = oracle_mod.normalize(c.points)
    x = x.astype(np.float64)
    area = np.full(len(x), 4.0 * np.pi * (np.linalg.norm(x, axis=1).mean() ** 2) / len(x))
    mu = iterate.orient(x, iters=10, backend="direct", areas=area)
    assert np.allclose(np.linalg.norm(mu, axis=1), area, rtol=1e-12)
    assert np.all((mu * x).sum(1) > 0)


# ---------------------------------------- kNN local areas (Sec. 6.1, Table 5)

def _areas_part(args):
    from oracle.areas import knn_areas
    x, nbr, rows = args
    return knn_areas(x, rows=rows, nbr=nbr)


def test_knn_areas_reproduce_table5():
    """Table 5, kNN column: the estimate on the 163,842-vertex unit sphere
    has the printed min, max, mean and total (4 significant digits)."""
    import os
    from concurrent.futures import ProcessPoolExecutor
    from oracle.areas import knn
    path = os.path.join(os.path.dirname(__file__), "golden", "table5_sphere_areas.txt")
    rows = {}
    for line in open(path):
        if line.startswith("#") or line.startswith("stat") or not line.strip():
            continue
        k, gt, kn, solved = line.split()
        rows[k] = float(kn)
    x = synth.icosphere(7).points.astype(np.float64)
    nbr = knn(x, 16)
    parts = np.array_split(np.arange(len(x)), 8)
    with ProcessPoolExecutor(8) as ex:
        a = np.concatenate(list(ex.map(_areas_part, [(x, nbr, p) for p in parts])))
    for stat, v in (("min", a.min()), ("max", a.max()), ("mean", a.mean()), ("total", a.sum())):
        assert abs(v / rows[stat] - 1) < 1e-3, (stat, v, rows[stat])


def _rotation(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    return q


def test_knn_areas_lattices_by_hand():
    """Planar lattices, rotated and shifted: an interior point of a square
    lattice of spacing a has the cell a^2, of a triangular lattice
    (sqrt(3)/2) a^2; the corner of a 5 x 5 square grid of spacing 1 has the
    quadrant cell [-R, 1/2]^2 with R = 4 (its 16th neighbour is at (4, 0)):
    area 4.5^2."""
    from oracle.areas import knn_areas
    a = 0.03
    R = _rotation(4)
    shift = np.array([0.1, -0.2, 0.05])
    g = np.arange(-4, 5)
    sq = np.array([(i, j, 0.0) for i in g for j in g]) * a
    centre = int(np.where((sq == 0).all(1))[0][0])
    out = knn_areas(sq @ R.T + shift)
    assert abs(out[centre] / a ** 2 - 1) < 1e-9
    tri = np.array([(i + 0.5 * (j % 2), j * np.sqrt(3) / 2, 0.0) for i in g for j in g]) * a
    c2 = int(np.argmin(np.linalg.norm(tri - tri.mean(0), axis=1)))
    out = knn_areas(tri @ R.T + shift)
    assert abs(out[c2] / (np.sqrt(3) / 2 * a * a) - 1) < 1e-9
    g5 = np.arange(5)
    grid = np.array([(i, j, 0.0) for i in g5 for j in g5])
    out = knn_areas(grid @ R.T)
    assert abs(out[0] - 4.5 ** 2) < 1e-9


def test_knn_areas_tiny_clouds():
    """Three points (0,0), (1,0), (0,2): the first has the cell
    {x <= 1/2, y <= 1} clipped to [-2, 2]^2 (R = 2, e1 along (1,0)), area
    2.5 * 3; clouds of one or two points have no plane and get 0; the
    estimate scales with the square of a uniform scale."""
    from oracle.areas import knn_areas
    P = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 2.0, 0.0]])
    out = knn_areas(P @ _rotation(7).T)
    assert abs(out[0] - 7.5) < 1e-9
    assert np.all(knn_areas(P[:2]) == 0) and np.all(knn_areas(P[:1]) == 0)
    x = synth.fibonacci_sphere(400, 2).points.astype(np.float64)
    assert np.allclose(knn_areas(3.0 * x), 9.0 * knn_areas(x), rtol=1e-9)
    assert np.all(knn_areas(x) > 0)


# ------------------------- far-field extension: Taylor orders, cutoff-safe test

def test_far_field_taylor_orders_converge_at_their_rate(oracle_mod):
    """A cluster accepted as one node by far targets: the error of the order-p
    far field against the exact sum falls by 2^(p+1) when the cluster shrinks
    by 2 (p = 0: the representative term, whose x_B cancels no first moment
    of random vectors; p = 1, 2: the Taylor terms).  A wrong sign, index or
    factor in a term of order p leaves an error of that order and breaks the
    rate."""
    rng = np.random.default_rng(1)
    base = rng.standard_normal((12, 3)) * 0.05
    mu = synth.random_unit(rng, 12) * 0.01
    rho = rng.uniform(-1, 1, 12)
    tg = np.array([[0.9, 0.7, -0.6], [-0.8, 0.9, 0.85]])
    want = {0: (1.7, 2.4), 1: (3.3, 4.7), 2: (6.5, 9.5)}
    for op, nu in (("A", mu), ("AT", rho), ("G", mu)):
        prev = None
        for order in (0, 1, 2):
            errs = []
            for s_ in (0.5, 0.25):
                x = base * s_ + np.array([0.1, -0.05, 0.02])
                t = oracle_mod.Tree(x).apply(op, nu, 0.0, 0.3, targets=tg, order=order)
                ex = oracle_mod.direct(op, x, nu, 0.0, targets=tg)
                errs.append(np.linalg.norm(t - ex) / np.linalg.norm(ex))
            lo, hi = want[order]
            assert lo < errs[0] / errs[1] < hi, (op, order, errs)
            if prev is not None:
                assert errs[1] < prev
            prev = errs[1]


def test_far_field_of_coincident_sources_is_the_representative(oracle_mod):
    """Sources at one location: every moment about x_B is 0, so orders 1 and 2
    equal order 0 (and the exact sum)."""
    rng = np.random.default_rng(2)
    x = np.repeat(np.array([[0.2, -0.1, 0.3]]), 5, axis=0)
    mu = synth.random_unit(rng, 5)
    tg = np.array([[-0.7, 0.8, -0.9]])
    for op, nu in (("A", mu), ("AT", rng.uniform(-1, 1, 5)), ("G", mu)):
        T = oracle_mod.Tree(x, max_depth=3)
        r0 = T.apply(op, nu, 0.0, 0.3, targets=tg)
        for order in (1, 2):
            assert np.allclose(T.apply(op, nu, 0.0, 0.3, targets=tg, order=order), r0,
                               rtol=1e-14, atol=0)
        assert np.allclose(r0, oracle_mod.direct(op, x, nu, 0.0, targets=tg), rtol=1e-12)


def test_cutoff_safe_acceptance_restores_the_cutoff(oracle_mod):
    """On a dense 20k cloud most targets have points within w = 0.002, which
    Alg. 4's representatives carry although the exact sum drops them: the
    gradient error stays at a few 1e-2 whatever the order.  Accepting only
    nodes whose cell is beyond w removes that error; with order 2 the
    remaining Taylor error is below 1e-3."""
    rng = np.random.default_rng(3)
    c = synth.torus_knot(20000, 5, with_init=False)
    x, _, sc = oracle_mod.normalize(c.points)
    nrm = np.nan_to_num(c.normals)
    bad = ~np.isfinite(c.normals).all(1)
    nrm[bad] = synth.random_unit(rng, int(bad.sum()))
    mu = nrm * c.area * sc * sc / c.n
    T = oracle_mod.Tree(x)
    ex = oracle_mod.direct("G", x, mu, 0.002)

    def err(order, ws):
        g = T.apply("G", mu, 0.002, 2.0, order=order, wsafe=ws)
        return np.linalg.norm(g - ex) / np.linalg.norm(ex)

    plain, safe2 = err(0, False), err(2, True)
    assert plain > 1e-2 and err(2, False) > 1e-2
    assert err(0, True) < 0.2 * plain
    assert safe2 < 1e-3


# -------------------- position gradients of the winding number (extension)

def test_winding_grad_x_matches_finite_differences(oracle_mod):
    """dL/dx of L = g . A(mu) from the closed form (-g G + P) against central
    differences of the exact sums, on a random cloud with no pair near the
    cutoff; the gradient sums to 0 (L is translation invariant)."""
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, (60, 3))
    mu = rng.standard_normal((60, 3))
    g = rng.standard_normal(60)
    for w in (0.0, 0.05):
        d = np.linalg.norm(x[:, None] - x[None], axis=2) + 10.0 * np.eye(len(x))
        assert np.all(np.abs(d - w) > 1e-3)  # no pair within the FD step of w
        gx = oracle_mod.winding_grad_x(x, mu, g, w)
        h = 1e-6
        fd = np.zeros_like(x)
        for k in range(len(x)):
            for a in range(3):
                xp, xm = x.copy(), x.copy()
                xp[k, a] += h
                xm[k, a] -= h
                fd[k, a] = (g @ oracle_mod.direct("A", xp, mu, w)
                            - g @ oracle_mod.direct("A", xm, mu, w)) / (2 * h)
        assert np.abs(gx - fd).max() <= 1e-7 * np.abs(fd).max()
        assert np.abs(gx.sum(axis=0)).max() <= 1e-12 * np.abs(gx).max()


def test_winding_grad_x_two_points_by_hand(oracle_mod):
    """x1 = 0, x2 = (1,0,0), mu1 = (1,0,0), mu2 = 0, g = (0,1): L = s_2 =
    -(x2 - x1).mu1 / (4 pi |x2 - x1|^3), so dL/dx2 = (1/(2 pi), 0, 0) and
    dL/dx1 = -dL/dx2."""
    x = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    mu = np.array([[1.0, 0, 0], [0.0, 0, 0]])
    g = np.array([0.0, 1.0])
    gx = oracle_mod.winding_grad_x(x, mu, g, 0.0)
    assert np.allclose(gx[1], [1 / (2 * np.pi), 0, 0], rtol=1e-14, atol=1e-16)
    assert np.allclose(gx[0], -gx[1], rtol=1e-14, atol=1e-16)


def test_winding_grad_x_treecode_limits(oracle_mod):
    """The treecode's position gradient equals the exact one when no node is
    accepted (c -> infinity) and approaches it at c = 2."""
    rng = np.random.default_rng(4)
    c = synth.fibonacci_sphere(1500, 1)
    x, _, sc = oracle_mod.normalize(c.points)
    mu = c.normals * (4 * np.pi * sc * sc / c.n)
    g = rng.standard_normal(c.n)
    ex = oracle_mod.winding_grad_x(x, mu, g, 0.002)
    T = oracle_mod.Tree(x)
    big = oracle_mod.winding_grad_x(x, mu, g, 0.002, backend="tree", c=1e6, tree=T)
    assert np.abs(big - ex).max() <= 1e-12 * np.abs(ex).max()
    tc = oracle_mod.winding_grad_x(x, mu, g, 0.002, backend="tree", c=2.0, tree=T)
    assert np.linalg.norm(tc - ex) / np.linalg.norm(ex) < 0.05


def test_gradient_grad_x_matches_finite_differences(oracle_mod):
    """dL/dx of L = v . grad F(mu) = -v . G(mu) from the closed form
    T(mu; v) + T(v; mu) against central differences of the exact sums; it
    sums to 0 (translation invariance); the treecode version equals it when
    no node is accepted."""
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, (50, 3))
    mu = rng.standard_normal((50, 3))
    v = rng.standard_normal((50, 3))
    for w in (0.0, 0.05):
        d = np.linalg.norm(x[:, None] - x[None], axis=2) + 10.0 * np.eye(len(x))
        assert np.all(np.abs(d - w) > 1e-3)
        gx = oracle_mod.gradient_grad_x(x, mu, v, w)
        h = 1e-6
        fd = np.zeros_like(x)
        for k in range(len(x)):
            for a in range(3):
                xp, xm = x.copy(), x.copy()
                xp[k, a] += h
                xm[k, a] -= h
                fd[k, a] = ((v * -oracle_mod.direct("G", xp, mu, w)).sum()
                            - (v * -oracle_mod.direct("G", xm, mu, w)).sum()) / (2 * h)
        assert np.abs(gx - fd).max() <= 1e-7 * np.abs(fd).max()
        assert np.abs(gx.sum(axis=0)).max() <= 1e-12 * np.abs(gx).max()
        big = oracle_mod.gradient_grad_x(x, mu, v, w, backend="tree", c=1e6)
        assert np.abs(big - gx).max() <= 1e-12 * np.abs(gx).max()


# ------------------------------------- leaves of more than one point (extension)

def test_leaf_capacity_tree_invariants(oracle_mod):
    """With leaf capacity K every leaf holds at most K points (or sits at the
    depth limit), every internal node more than K, children partition their
    parent; K >= N leaves the root alone, and then the treecode is the exact
    sum (no target in [-1,1]^3 is farther than c * 2 = 4 from x_B)."""
    rng = np.random.default_rng(8)
    x = rng.uniform(-0.9, 0.9, (700, 3))
    x[:40] = x[0]  # coincident points beyond every K below
    for K in (2, 8, 33):
        T = oracle_mod.Tree(x, leaf_cap=K)
        d, leaf, b, e, order = T.export()
        cnt = e - b
        assert np.all((cnt[leaf == 1] <= K) | (d[leaf == 1] == 15))
        assert np.all(cnt[leaf == 0] > K)
        assert np.all(cnt[leaf == 1] >= 1)
        # the leaves partition the points
        assert np.array_equal(np.sort(np.concatenate([order[bb:ee] for bb, ee, l in
                                                     zip(b, e, leaf) if l])), np.arange(len(x)))
    T = oracle_mod.Tree(x, leaf_cap=len(x))
    assert T.nnodes == 1
    mu = rng.standard_normal((len(x), 3))
    for op, nu in (("A", mu), ("G", mu), ("AT", rng.standard_normal(len(x)))):
        tc = T.apply(op, nu, 0.01, 2.0)
        ex = oracle_mod.direct(op, x, nu, 0.01)
        assert np.allclose(tc, ex, rtol=1e-12, atol=1e-12 * np.abs(ex).max())

