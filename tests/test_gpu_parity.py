"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

* normalization: bit-identical FP32 coordinates;
* octree: identical node sets (depth and member points), bit-exact;
* moments: per node, FP32 rounding of the FP64 sums;
* operators A, A^T, G: per target against the oracle treecode with the same
  (c, D, w), at the FP32 tolerance below, plus pair counts;
* Alg. 3: flip rate of the final normals against the oracle's run.

The bar of one operator call (per target 1e-5 of the summed term
magnitudes, exemptions only for oracle-reported decision near-ties and at
most 1e-4 of targets, relative L2 and pair counts) is `parity_bar.check`.
"""
import numpy as np
import pytest

import parity_bar
import synth

pytestmark = pytest.mark.gpu

TOL = parity_bar.TOL


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_16634_amd as w
    w.load_library()
    return torch.device("cuda:0")


def _cloud(name):
    if name == "sphere2k":
        c = synth.fibonacci_sphere(2000, 0)
        return c, 0.002, 0.016
    if name == "ellipsoids50k":
        c = synth.ellipsoid_union(50000, 2)
        return c, 0.02, 0.08
    if name == "ragged3077":
        c = synth.ellipsoid_union(3077, 9, noise=0.001)
        return c, 0.002, 0.016
    if name == "knot20k":
        c = synth.torus_knot(20000, 5)
        return c, 0.002, 0.016
    raise KeyError(name)


def _to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def _node_sets(depth, begin, end, order):
    return {(int(d), tuple(sorted(order[b:e].tolist()))) for d, b, e in zip(depth, begin, end)}


def _setup(dev, cloud, c=2.0, depth=15):
    import paper_2405_16634_amd as w
    import oracle
    ctx = w.Context(0)
    P = _to_dev(cloud.points, dev)
    x_dev, norm = ctx.normalize(P)
    x_or, ctr, sc = oracle.normalize(cloud.points)
    ctx.build(x_dev, c, depth)
    return ctx, x_dev, x_or, sc, norm


CASES = ["sphere2k", "ragged3077", "knot20k", "ellipsoids50k"]


@pytest.mark.parametrize("name", CASES)
def test_normalize_and_tree_are_identical(dev, name, oracle_mod):
    cloud, _, _ = _cloud(name)
    print(f"[case] {name} n={cloud.n}", flush=True)
    ctx, x_dev, x_or, sc, norm = _setup(dev, cloud)
    x_gpu = x_dev.cpu().numpy()
    assert np.array_equal(x_gpu, x_or), "normalized coordinates differ"
    assert abs(norm.scale - sc) <= 1e-15 * sc
    d, leaf, b, e, perm = ctx.tree()
    T = oracle_mod.Tree(x_or.astype(np.float64))
    od, ol, obg, oen, oorder = T.export()
    assert len(d) == T.nnodes
    g_sets = _node_sets(d, b, e, perm)
    o_sets = _node_sets(od, obg, oen, oorder)
    assert g_sets == o_sets
    # leaves: one point or at the depth limit, as in the oracle
    gl = {(int(dd), tuple(sorted(perm[bb:ee].tolist()))) for dd, l, bb, ee in zip(d, leaf, b, e) if l}
    ol_ = {(int(dd), tuple(sorted(oorder[bb:ee].tolist()))) for dd, l, bb, ee in zip(od, ol, obg, oen) if l}
    assert gl == ol_
    # pre-order: the first child of an internal node is the next node and
    # ranges nest
    inner = np.where(leaf == 0)[0]
    assert np.all(d[inner + 1] == d[inner] + 1)
    assert np.all(b[inner + 1] == b[inner])
    ctx.close()


def test_tree_edge_cases(dev, oracle_mod):
    import paper_2405_16634_amd as w
    rng = np.random.default_rng(4)
    cases = {
        "single": np.array([[0.25, -0.5, 0.75]], np.float32),
        "pair": np.array([[0.1, 0.1, 0.1], [0.2, 0.1, 0.1]], np.float32),
        "duplicates": np.repeat(rng.uniform(-0.9, 0.9, (7, 3)).astype(np.float32), 5, axis=0),
        "split_plane": np.array([[0, 0, 0], [-1e-12, 0, 0], [0.5, 0.5, 0.5], [1, 1, 1], [-1, -1, -1]],
                                np.float32),
        "ragged_257": rng.uniform(-1, 1, (257, 3)).astype(np.float32),
    }
    for name, x in cases.items():
        print(f"[case] tree edge {name}", flush=True)
        for depth in (15, 4):
            ctx = w.Context(0)
            ctx.build(_to_dev(x, dev), 2.0, depth)
            d, leaf, b, e, perm = ctx.tree()
            T = oracle_mod.Tree(x.astype(np.float64), max_depth=depth)
            od, ol, obg, oen, oorder = T.export()
            assert _node_sets(d, b, e, perm) == _node_sets(od, obg, oen, oorder), (name, depth)
            ctx.close()


@pytest.mark.parametrize("name", ["sphere2k", "knot20k"])
def test_moments_match(dev, name, oracle_mod):
    import torch
    cloud, _, _ = _cloud(name)
    ctx, x_dev, x_or, sc, _ = _setup(dev, cloud)
    rng = np.random.default_rng(12)
    mu = (synth.random_unit(rng, cloud.n) * (cloud.area * sc * sc / cloud.n)).astype(np.float32)
    rho = rng.standard_normal(cloud.n).astype(np.float32)
    d, leaf, b, e, perm = ctx.tree()
    T = oracle_mod.Tree(x_or.astype(np.float64))
    od, ol, obg, oen, oorder = T.export()
    key_o = {(int(dd), tuple(sorted(oorder[bb:ee].tolist()))): k for k, (dd, bb, ee) in enumerate(zip(od, obg, oen))}
    idx = np.array([key_o[(int(dd), tuple(sorted(perm[bb:ee].tolist())))] for dd, bb, ee in zip(d, b, e)])
    for nu in (mu, rho):
        xB, nuB, W = ctx.moments(_to_dev(nu, dev))
        oxB, onuB, oW = T.reps(nu.astype(np.float64))
        oxB, onuB, oW = oxB[idx], onuB[idx], oW[idx]
        assert np.allclose(W, oW, rtol=2e-7, atol=0)
        ok = oW > 0
        assert np.max(np.abs(xB[ok] - oxB[ok])) <= 1.2e-7
        scale = np.abs(onuB).max()
        assert np.max(np.abs(nuB - onuB)) <= 1e-6 * scale
    ctx.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("name", CASES)
def test_operators_match_oracle_treecode(dev, name, oracle_mod):
    import paper_2405_16634_amd as w
    import torch
    cloud, w1, w2 = _cloud(name)
    print(f"[case] operators {name} n={cloud.n}", flush=True)
    ctx, x_dev, x_or, sc, _ = _setup(dev, cloud)
    T = oracle_mod.Tree(x_or.astype(np.float64))
    rng = np.random.default_rng(7)
    sigma = np.full(cloud.n, cloud.area * sc * sc / cloud.n, np.float32)
    nrm = synth.random_unit(rng, cloud.n).astype(np.float32)
    rho = (0.5 - rng.uniform(0, 1, cloud.n)).astype(np.float32)
    mu = nrm * sigma[:, None]
    ctx.set_flags(w.FLAG_COUNT_PAIRS)
    for w_ in (w1, w2):
        runs = {}
        # the default walk (sparse subtrees deferred) and the lockstep walk
        for defer in (ctx.defer(), 0):
            ctx.set_defer(defer)
            ctx.reset_stats()
            s = ctx.winding(_to_dev(nrm, dev), w_, sigma=_to_dev(sigma, dev)).cpu().numpy()
            g = ctx.gradient(_to_dev(mu, dev), w_).cpu().numpy()
            at = ctx.adjoint(_to_dev(rho, dev), w_).cpu().numpy()
            runs[defer] = (s, g, at, ctx.stats())
        ctx.set_defer(32)
        for op, nu, sign in (("A", mu.astype(np.float64), 1.0),
                             ("G", mu.astype(np.float64), -1.0),
                             ("AT", rho.astype(np.float64), 1.0)):
            ref, mag, pairs, mg = T.apply(op, nu, w_, 2.0, with_stats=True, with_margins=True)
            ref = sign * ref  # the library returns grad F = -G
            k = {"A": 0, "AT": 1, "G": 2}[op]
            for defer, (s, g, at, st) in runs.items():
                got = {"A": s, "G": g, "AT": at}[op]
                r = parity_bar.check(f"{name} {op} w={w_} defer={defer}", got, ref, mag, mg,
                                     pairs_gpu=st["pairs"][k], pairs_oracle=pairs)
                print(f"  {op} w={w_} defer={defer}: {parity_bar.fmt(r)}", flush=True)
    ctx.close()
    torch.cuda.synchronize()


def test_direct_limit_matches_exact_sums(dev, oracle_mod):
    """With c huge every node is opened: the treecode is the exact sum."""
    cloud, w1, _ = _cloud("sphere2k")
    import paper_2405_16634_amd as w
    ctx, x_dev, x_or, sc, _ = _setup(dev, cloud, c=1e6)
    rng = np.random.default_rng(3)
    mu = (synth.random_unit(rng, cloud.n) * (4 * np.pi * sc * sc / cloud.n)).astype(np.float32)
    s = ctx.winding(_to_dev(mu, dev), w1).cpu().numpy()
    ref, mag = oracle_mod.direct("A", x_or, mu, w1, with_mag=True)
    rel = np.abs(s - ref) / mag
    assert rel.max() < TOL
    ctx.close()


@pytest.mark.parametrize("name", ["sphere2k", "ragged3077", "knot20k"])
def test_orient_matches_oracle(dev, name, oracle_mod):
    import torch
    cloud, w1, w2 = _cloud(name)
    print(f"[case] orient {name} n={cloud.n}", flush=True)
    ctx, x_dev, x_or, sc, _ = _setup(dev, cloud)
    mu_g = ctx.orient(40, w1, w2).cpu().numpy().astype(np.float64)
    E = ctx.energy(40)
    mu_o = oracle_mod.orient(x_or, iters=40, w1=w1, w2=w2, backend="tree")
    dots = (mu_g * mu_o).sum(1)
    flip = (dots <= 0).mean()
    ng = mu_g / np.linalg.norm(mu_g, axis=1, keepdims=True)
    no = mu_o / np.linalg.norm(mu_o, axis=1, keepdims=True)
    ang = np.degrees(np.arccos(np.clip((ng * no).sum(1), -1, 1)))
    print(f"  flip={flip:.2e} mean_angle={ang.mean():.3e} deg E0={E[0]:.3e} E39={E[-1]:.3e}", flush=True)
    assert flip <= 1e-3
    assert E[0] == pytest.approx(0.25 * cloud.n)
    ctx.close()
    torch.cuda.synchronize()


def test_orient_resume_is_exact(dev):
    """Stopping after iteration 17 of 40 and resuming at 18 with the returned
    mu reproduces the uninterrupted run bit for bit: (mu, i) is the state."""
    cloud, w1, w2 = _cloud("ragged3077")
    ctx, x_dev, x_or, sc, _ = _setup(dev, cloud)
    full = ctx.orient(40, w1, w2).clone()
    again = ctx.orient(40, w1, w2).clone()
    assert bool((full == again).all()), "orient is not deterministic"
    half = ctx.orient(40, w1, w2, stop_iter=17).clone()
    rest = ctx.orient(40, w1, w2, mu0=half, start_iter=18).clone()
    assert bool((rest == full).all())
    ctx.close()
