"""Extensions in combination, against the oracle or against each other:
the far field of order 2 and leaves of several points on a batched forest,
queries and the neighbour search on a tree with leaves of several points.
The per-target bar is the operator bar (`parity_bar.check`: |error| <= 1e-5
of the summed term magnitudes, exemptions only for oracle-reported decision
near-ties).
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


@pytest.mark.parametrize("order,wsafe,K", [(2, True, 1), (0, False, 8), (2, True, 8)])
def test_batched_forest_matches_oracle_per_cloud(dev, order, wsafe, K, oracle_mod):
    import torch
    import paper_2405_16634_amd as w
    import oracle
    clouds = [synth.fibonacci_sphere(2000, 0).points,
              synth.ellipsoid_union(3077, 9, noise=0.001, with_init=False).points,
              np.repeat(np.random.default_rng(3).uniform(-1, 1, (4, 3)).astype(np.float32), 3, 0)]
    off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])]).astype(np.int64)
    print(f"[case] batched order={order} wsafe={wsafe} K={K}", flush=True)
    ctx = w.Context(0)
    x, _ = ctx.normalize_batched(torch.from_numpy(np.concatenate(clouds)).to(dev), off)
    ctx.build_batched(x, off, 2.0, 15, K)
    ctx.set_far_field(order, wsafe)
    rng = np.random.default_rng(11)
    mu = (synth.random_unit(rng, int(off[-1])) * 1e-3).astype(np.float32)
    rho = (0.5 - rng.uniform(0, 1, int(off[-1]))).astype(np.float32)
    got = {"A": ctx.winding(_t(mu, dev), 0.002).cpu().numpy(),
           "G": -ctx.gradient(_t(mu, dev), 0.002).cpu().numpy(),
           "AT": ctx.adjoint(_t(rho, dev), 0.002).cpu().numpy()}
    for c, pts in enumerate(clouds):
        a, b = off[c], off[c + 1]
        x_or, _, _ = oracle.normalize(pts)
        T = oracle_mod.Tree(x_or, leaf_cap=K)
        for op, nu in (("A", mu), ("G", mu), ("AT", rho)):
            ref, mag, _, mg = T.apply(op, nu[a:b].astype(np.float64), 0.002, 2.0,
                                      with_stats=True, order=order, wsafe=wsafe,
                                      with_margins=True)
            r = parity_bar.check(f"batched order={order} K={K} cloud {c} {op}", got[op][a:b],
                                 ref, mag, mg)
            print(f"  cloud {c} {op}: {parity_bar.fmt(r)}", flush=True)
    ctx.close()


def test_queries_on_leaves_of_several_points(dev, oracle_mod):
    import paper_2405_16634_amd as w
    import oracle
    cloud = synth.torus_knot(20000, 5, with_init=False)
    print("[case] queries K=8 knot20k", flush=True)
    ctx = w.Context(0)
    x, _ = ctx.normalize(_t(cloud.points, dev))
    x_or, _, sc = oracle.normalize(cloud.points)
    ctx.build(x, 2.0, 15, 8)
    rng = np.random.default_rng(12)
    mu = (synth.random_unit(rng, cloud.n) * (cloud.area * sc * sc / cloud.n)).astype(np.float32)
    Q = rng.uniform(-1, 1, (2001, 3)).astype(np.float32)
    Q[:400] = x_or[:400] + 1e-3 * rng.standard_normal((400, 3))
    got = ctx.winding_at(_t(mu, dev), 0.002, _t(Q, dev)).cpu().numpy()
    ref, mag, _, mg = oracle_mod.Tree(x_or, leaf_cap=8).apply(
        "A", mu.astype(np.float64), 0.002, 2.0, targets=Q.astype(np.float64), with_stats=True,
        with_margins=True)
    r = parity_bar.check("queries K=8", got, ref, mag, mg)
    print(f"  {parity_bar.fmt(r)}", flush=True)
    ctx.close()


def test_neighbour_search_does_not_depend_on_the_leaves(dev):
    """The 16 nearest neighbours are a property of the points: the same on
    trees with single-point leaves and with leaves of up to 8 or 64 points."""
    import paper_2405_16634_amd as w
    cloud = synth.torus_knot(50000, 5, with_init=False)
    print("[case] kNN vs leaf capacity knot50k", flush=True)
    res = []
    for K in (1, 8, 64):
        ctx = w.Context(0)
        x, _ = ctx.normalize(_t(cloud.points, dev))
        ctx.build(x, 2.0, 15, K)
        _, nbr = ctx.features(with_neighbours=True)
        res.append(nbr.cpu().numpy())
        ctx.close()
    assert np.array_equal(res[0], res[1]) and np.array_equal(res[0], res[2])


def test_prefetch_is_bit_identical_with_far_field_and_leaf_capacity(dev):
    """The prefetch setting changes no bit, also with the far field of order
    2 (which keeps the plain record loads) and with leaves of several points
    (direct sums inside the prefetching walk)."""
    import paper_2405_16634_amd as w
    cloud = synth.torus_knot(20000, 5, with_init=False)
    print("[case] prefetch x far field x leaf capacity knot20k", flush=True)
    rng = np.random.default_rng(13)
    mu = _t(synth.random_unit(rng, cloud.n) * 1e-4, dev)
    rho = _t(0.5 - rng.uniform(0, 1, cloud.n), dev)
    for K, order in ((1, 2), (8, 0), (8, 2)):
        ctx = w.Context(0)
        x, _ = ctx.normalize(_t(cloud.points, dev))
        ctx.build(x, 2.0, 15, K)
        ctx.set_far_field(order, order > 0)
        ctx.set_defer(0)  # the lockstep walk in both prefetch settings
        res = []
        for pf in (False, True):
            ctx.set_prefetch(pf)
            res.append((ctx.winding(mu, 0.002).clone(), ctx.gradient(mu, 0.002).clone(),
                        ctx.adjoint(rho, 0.002).clone(), ctx.orient(5, 0.002, 0.016).clone()))
        for a, b in zip(*res):
            assert bool((a == b).all()), (K, order)
        ctx.close()
