"""Position gradients of the winding number (an extension: differentiable
winding numbers in the points) on the HIP path against the FP64 oracle.

dL/dx_k of L = sum_i g_i A_w(mu)_i is g_k grad F(x_k) + p_k with p one more
treecode walk (scalar sources g, each target with its own mu_k).  Parity per
target against the oracle's treecode with the same (c, D): |error| <= 1e-5
of the sum of the term magnitudes of both parts (`parity_bar.check`:
exemptions only for oracle-reported decision near-ties in either walk); with
every node opened (c =
1e6) against the exact sums.  The closed form itself is pinned on the CPU
(finite differences, translation invariance, a two-point hand value).
"""
import numpy as np
import pytest

import parity_bar
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_16634_amd as w
    w.load_library()
    return torch.device("cuda:0")


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def _setup(dev, cloud, c=2.0):
    import paper_2405_16634_amd as w
    import oracle
    ctx = w.Context(0)
    x_dev, _ = ctx.normalize(_t(cloud.points, dev))
    x_or, _, sc = oracle.normalize(cloud.points)
    ctx.build(x_dev, c, 15)
    return ctx, x_dev, x_or, sc


def _inputs(cloud, sc, seed):
    rng = np.random.default_rng(seed)
    mu = (synth.random_unit(rng, cloud.n) * (cloud.area * sc * sc / cloud.n)).astype(np.float32)
    g = rng.standard_normal(cloud.n).astype(np.float32)
    return mu, g


def _check(got, x_or, mu, g, w, c, oracle_mod):
    T = oracle_mod.Tree(x_or)
    m64, g64 = mu.astype(np.float64), g.astype(np.float64)
    G, magG, _, mgG = T.apply("G", m64, w, c, with_stats=True, with_margins=True)
    P, magP, _, mgP = T.apply("P", g64, w, c, with_stats=True, tvec=m64, with_margins=True)
    ref = -g64[:, None] * G + P
    mag = np.abs(g64) * magG + magP
    r = parity_bar.check(f"winding_grad_x w={w} c={c}", got, ref, mag, np.hstack([mgG, mgP]))
    print(f"  {parity_bar.fmt(r)}", flush=True)
    return ref


@pytest.mark.parametrize("name", ["sphere2k", "ragged3077", "knot20k"])
def test_winding_grad_x_matches_oracle_treecode(dev, name, oracle_mod):
    cloud = {"sphere2k": lambda: synth.fibonacci_sphere(2000, 0),
             "ragged3077": lambda: synth.ellipsoid_union(3077, 9, noise=0.001, with_init=False),
             "knot20k": lambda: synth.torus_knot(20000, 5, with_init=False)}[name]()
    print(f"[case] position gradient {name}", flush=True)
    ctx, _, x_or, sc = _setup(dev, cloud)
    mu, g = _inputs(cloud, sc, 21)
    for w_ in (0.002, 0.016):
        got = ctx.winding_grad_x(_t(mu, dev), w_, _t(g, dev)).cpu().numpy()
        _check(got, x_or, mu, g, w_, 2.0, oracle_mod)
    # the far-field setting does not change the position gradient
    ctx.set_far_field(2, True)
    again = ctx.winding_grad_x(_t(mu, dev), 0.016, _t(g, dev)).cpu().numpy()
    assert np.array_equal(again, got)
    ctx.close()


def test_winding_grad_x_exact_limit(dev, oracle_mod):
    """c = 1e6: every node is opened; the device equals the exact closed form."""
    cloud = synth.fibonacci_sphere(2000, 0)
    print("[case] position gradient exact limit", flush=True)
    ctx, _, x_or, sc = _setup(dev, cloud, c=1e6)
    mu, g = _inputs(cloud, sc, 22)
    got = ctx.winding_grad_x(_t(mu, dev), 0.002, _t(g, dev)).cpu().numpy().astype(np.float64)
    ref = oracle_mod.winding_grad_x(x_or, mu.astype(np.float64), g.astype(np.float64), 0.002)
    _check(got, x_or, mu, g, 0.002, 1e6, oracle_mod)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5
    ctx.close()


def test_autograd_in_positions(dev, oracle_mod):
    """winding_at_points: backward in x is the position gradient and in mu
    the adjoint; the sum of x.grad is about 0 (translation invariance, up to
    the treecode's error)."""
    import torch
    import paper_2405_16634_amd as w
    from paper_2405_16634_amd.autograd import winding_at_points
    cloud = synth.ellipsoid_union(3077, 9, noise=0.001, with_init=False)
    print("[case] position gradient autograd", flush=True)
    ctx, x_dev, x_or, sc = _setup(dev, cloud)
    mu, g = _inputs(cloud, sc, 23)
    x = x_dev.clone().requires_grad_(True)
    m = _t(mu, dev).requires_grad_(True)
    s = winding_at_points(ctx, x, m, 0.002)
    (s * _t(g, dev)).sum().backward()
    gx = ctx.winding_grad_x(_t(mu, dev), 0.002, _t(g, dev))
    gm = ctx.adjoint(_t(g, dev), 0.002)
    assert torch.equal(x.grad, gx) and torch.equal(m.grad, gm)
    ref = _check(x.grad.cpu().numpy(), x_or, mu, g, 0.002, 2.0, oracle_mod)
    tot = np.abs(x.grad.cpu().numpy().astype(np.float64).sum(0)).max()
    assert tot < 1e-2 * np.abs(ref).sum(0).max()
    with pytest.raises(ValueError):
        ctx.winding_grad_x(_t(mu, dev), 0.002, _t(g[:-1], dev))
    del w
    ctx.close()


def test_batched_matches_standalone(dev):
    """Two clouds in one forest: each cloud's position gradient equals its
    standalone value (walks never cross clouds)."""
    import torch
    import paper_2405_16634_amd as w
    clouds = [synth.fibonacci_sphere(2000, 0).points,
              synth.ellipsoid_union(3077, 9, noise=0.001, with_init=False).points]
    off = np.array([0, len(clouds[0]), len(clouds[0]) + len(clouds[1])], np.int64)
    print("[case] position gradient batched", flush=True)
    ctx = w.Context(0)
    P = torch.from_numpy(np.concatenate(clouds)).to(dev)
    x, _ = ctx.normalize_batched(P, off)
    ctx.build_batched(x, off)
    rng = np.random.default_rng(24)
    mu = (synth.random_unit(rng, len(P)) * 1e-3).astype(np.float32)
    g = rng.standard_normal(len(P)).astype(np.float32)
    got = ctx.winding_grad_x(_t(mu, dev), 0.002, _t(g, dev)).cpu().numpy()
    for c in range(2):
        lo, hi = off[c], off[c + 1]
        one = w.Context(0)
        xs, _ = one.normalize(torch.from_numpy(clouds[c]).to(dev))
        one.build(xs, 2.0, 15)
        ref = one.winding_grad_x(_t(mu[lo:hi], dev), 0.002, _t(g[lo:hi], dev)).cpu().numpy()
        err = np.abs(got[lo:hi] - ref).max() / np.abs(ref).max()
        print(f"  cloud {c}: max rel diff {err:.2e}", flush=True)
        assert err < 1e-5
        one.close()
    ctx.close()


# ---------------------- position gradient of grad F (third derivatives of Phi)

def _check_t(got, x_or, mu, v, w, c, oracle_mod):
    T = oracle_mod.Tree(x_or)
    m64, v64 = mu.astype(np.float64), v.astype(np.float64)
    t1, mag1, _, mg1 = T.apply("T", m64, w, c, with_stats=True, tvec=v64, with_margins=True)
    t2, mag2, _, mg2 = T.apply("T", v64, w, c, with_stats=True, tvec=m64, with_margins=True)
    ref = t1 + t2
    r = parity_bar.check(f"gradient_grad_x w={w} c={c}", got, ref, mag1 + mag2,
                         np.hstack([mg1, mg2]))
    print(f"  {parity_bar.fmt(r)}", flush=True)
    return ref


@pytest.mark.parametrize("name", ["sphere2k", "ragged3077", "knot20k"])
def test_gradient_grad_x_matches_oracle_treecode(dev, name, oracle_mod):
    cloud = {"sphere2k": lambda: synth.fibonacci_sphere(2000, 0),
             "ragged3077": lambda: synth.ellipsoid_union(3077, 9, noise=0.001, with_init=False),
             "knot20k": lambda: synth.torus_knot(20000, 5, with_init=False)}[name]()
    print(f"[case] grad F position gradient {name}", flush=True)
    ctx, _, x_or, sc = _setup(dev, cloud)
    mu, _ = _inputs(cloud, sc, 31)
    v = np.random.default_rng(32).standard_normal((cloud.n, 3)).astype(np.float32)
    for w_ in (0.002, 0.016):
        got = ctx.gradient_grad_x(_t(mu, dev), w_, _t(v, dev)).cpu().numpy()
        _check_t(got, x_or, mu, v, w_, 2.0, oracle_mod)
    ctx.close()


def test_gradient_grad_x_exact_limit_and_autograd(dev, oracle_mod):
    import torch
    from paper_2405_16634_amd.autograd import gradient_at_points
    cloud = synth.fibonacci_sphere(2000, 0)
    print("[case] grad F position gradient exact limit + autograd", flush=True)
    ctx, x_dev, x_or, sc = _setup(dev, cloud, c=1e6)
    mu, _ = _inputs(cloud, sc, 33)
    v = np.random.default_rng(34).standard_normal((cloud.n, 3)).astype(np.float32)
    got = ctx.gradient_grad_x(_t(mu, dev), 0.002, _t(v, dev)).cpu().numpy().astype(np.float64)
    ref = oracle_mod.gradient_grad_x(x_or, mu.astype(np.float64), v.astype(np.float64), 0.002)
    _check_t(got, x_or, mu, v, 0.002, 1e6, oracle_mod)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5
    # autograd at c = 2
    x = x_dev.clone().requires_grad_(True)
    m = _t(mu, dev).requires_grad_(True)
    gF = gradient_at_points(ctx, x, m, 0.002)
    (gF * _t(v, dev)).sum().backward()
    assert torch.equal(x.grad, ctx.gradient_grad_x(_t(mu, dev), 0.002, _t(v, dev)))
    assert torch.equal(m.grad, ctx.gradient(_t(v, dev), 0.002))
    _check_t(x.grad.cpu().numpy(), x_or, mu, v, 0.002, 2.0, oracle_mod)
    ctx.close()
