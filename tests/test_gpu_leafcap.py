"""Leaves of more than one point (an extension of the paper's tree, which
splits down to single points): the device octree, operators and Alg. 3
with a leaf capacity K against the oracle's tree with the same K.

* tree: identical sets of (depth, member points), leaves included (exact);
* operators: per target at the bar of the plain operators
  (`parity_bar.check`: |error| <= 1e-5 of the sum of term magnitudes,
  exemptions only for oracle-reported decision near-ties);
* Alg. 3: flip rate against the oracle's run <= 0.1 %;
* the approximation error against the exact sums shrinks as K grows.
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


def _cloud(name):
    return {"sphere2k": lambda: synth.fibonacci_sphere(2000, 0),
            "ragged3077": lambda: synth.ellipsoid_union(3077, 9, noise=0.001, with_init=False),
            "knot20k": lambda: synth.torus_knot(20000, 5, with_init=False)}[name]()


def _sets(depth, begin, end, order, leaf=None):
    return {(int(d), tuple(sorted(order[b:e].tolist())))
            for k, (d, b, e) in enumerate(zip(depth, begin, end)) if leaf is None or leaf[k]}


def _setup(dev, points, K, c=2.0, depth=15):
    import paper_2405_16634_amd as w
    import oracle
    ctx = w.Context(0)
    x_dev, _ = ctx.normalize(_t(points, dev))
    x_or, _, sc = oracle.normalize(points)
    ctx.build(x_dev, c, depth, K)
    return ctx, x_or, sc


@pytest.mark.parametrize("K", [2, 8, 32])
@pytest.mark.parametrize("name", ["sphere2k", "ragged3077", "knot20k"])
def test_tree_matches_oracle(dev, name, K, oracle_mod):
    cloud = _cloud(name)
    print(f"[case] leaf cap {K} tree {name}", flush=True)
    ctx, x_or, _ = _setup(dev, cloud.points, K)
    d, leaf, b, e, perm = ctx.tree()
    T = oracle_mod.Tree(x_or, leaf_cap=K)
    od, ol, obg, oen, oorder = T.export()
    assert len(d) == T.nnodes
    assert _sets(d, b, e, perm) == _sets(od, obg, oen, oorder)
    assert _sets(d, b, e, perm, leaf) == _sets(od, obg, oen, oorder, ol)
    assert np.all((e - b)[leaf == 1] <= K) or np.all(d[(leaf == 1) & (e - b > K)] == 15)
    inner = np.where(leaf == 0)[0]
    assert np.all(d[inner + 1] == d[inner] + 1) and np.all(b[inner + 1] == b[inner])
    ctx.close()


def test_tree_edge_cases(dev, oracle_mod):
    import paper_2405_16634_amd as w
    rng = np.random.default_rng(4)
    cases = {
        "single": np.array([[0.25, -0.5, 0.75]], np.float32),
        "duplicates": np.repeat(rng.uniform(-0.9, 0.9, (7, 3)).astype(np.float32), 5, axis=0),
        "ragged_257": rng.uniform(-1, 1, (257, 3)).astype(np.float32),
    }
    for name, x in cases.items():
        for depth in (15, 4):
            for K in (3, 64):
                print(f"[case] leaf cap {K} edge {name} D={depth}", flush=True)
                ctx = w.Context(0)
                ctx.build(_t(x, dev), 2.0, depth, K)
                d, leaf, b, e, perm = ctx.tree()
                T = oracle_mod.Tree(x.astype(np.float64), max_depth=depth, leaf_cap=K)
                od, ol, obg, oen, oorder = T.export()
                assert _sets(d, b, e, perm, leaf) == _sets(od, obg, oen, oorder, ol)
                assert _sets(d, b, e, perm) == _sets(od, obg, oen, oorder)
                ctx.close()
    ctx = w.Context(0)
    with pytest.raises(w.WnncError):
        ctx.build(_t(cases["ragged_257"], dev), 2.0, 15, 0)
    ctx.close()


@pytest.mark.parametrize("name", ["ragged3077", "knot20k"])
def test_operators_match_oracle(dev, name, oracle_mod):
    cloud = _cloud(name)
    K = 8
    print(f"[case] leaf cap {K} operators {name}", flush=True)
    ctx, x_or, sc = _setup(dev, cloud.points, K)
    T = oracle_mod.Tree(x_or, leaf_cap=K)
    rng = np.random.default_rng(7)
    mu = (synth.random_unit(rng, cloud.n) * (cloud.area * sc * sc / cloud.n)).astype(np.float32)
    rho = (0.5 - rng.uniform(0, 1, cloud.n)).astype(np.float32)
    for w_ in (0.002, 0.016):
        got = {"A": ctx.winding(_t(mu, dev), w_).cpu().numpy(),
               "G": -ctx.gradient(_t(mu, dev), w_).cpu().numpy(),
               "AT": ctx.adjoint(_t(rho, dev), w_).cpu().numpy()}
        for op, nu in (("A", mu), ("G", mu), ("AT", rho)):
            ref, mag, _, mg = T.apply(op, nu.astype(np.float64), w_, 2.0, with_stats=True,
                                      with_margins=True)
            r = parity_bar.check(f"leaf cap {K} {name} {op} w={w_}", got[op], ref, mag, mg)
            print(f"  {op} w={w_}: {parity_bar.fmt(r)}", flush=True)
    ctx.close()


def test_orient_matches_oracle(dev, oracle_mod):
    cloud = _cloud("ragged3077")
    print("[case] leaf cap 8 orient ragged3077", flush=True)
    ctx, x_or, _ = _setup(dev, cloud.points, 8)
    mu_g = ctx.orient(40, 0.01, 0.08).cpu().numpy().astype(np.float64)
    mu_o = oracle_mod.orient(x_or, iters=40, w1=0.01, w2=0.08, leaf_cap=8)
    flip = float(((mu_g * mu_o).sum(1) <= 0).mean())
    print(f"  flip={flip:.2e}", flush=True)
    assert flip <= 1e-3
    ctx.close()


def test_error_shrinks_with_leaf_capacity(dev, oracle_mod):
    """Gradient error against the exact sums, smooth mu, c = 2: bigger
    leaves sum more pairs exactly."""
    import oracle
    cloud = synth.ellipsoid_union(20000, 2, noise=0.0, with_init=False)
    print("[case] leaf cap accuracy ellipsoids20k", flush=True)
    x_or, _, sc = oracle.normalize(cloud.points)
    mu = (cloud.normals * (cloud.area * sc * sc / cloud.n)).astype(np.float32)
    exact = -oracle_mod.direct("G", x_or, mu.astype(np.float64), 0.002)
    errs = []
    for K in (1, 8, 32):
        ctx, _, _ = _setup(dev, cloud.points, K)
        g = ctx.gradient(_t(mu, dev), 0.002).cpu().numpy().astype(np.float64)
        errs.append(np.linalg.norm(g - exact) / np.linalg.norm(exact))
        print(f"  K={K}: grad rel-L2 {errs[-1]:.2e}", flush=True)
        ctx.close()
    assert errs[0] > errs[1] > errs[2]
