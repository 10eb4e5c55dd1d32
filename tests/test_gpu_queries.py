"""Winding number at query points off the surface (the field F of Sec. 3).

* every query matches the oracle's treecode at the same targets (Alg. 4 per
  query on the points' tree) at the operator bar of `parity_bar.check`;
* on the unit sphere with outward mu = n 4 pi / N, F is about 1 inside and
  about 0 outside (Thm. 1), and exactly the oracle's value at the centre;
* ragged query counts, a single query, queries far outside the root cell
  and queries coinciding with points (the cutoff) are covered;
* a batched tree is refused.
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


def _check(oracle_mod, xh, mu, Q, got, w_):
    T = oracle_mod.Tree(xh)
    ref, mag, _, mg = T.apply("A", mu.astype(np.float64), w_, 2.0, targets=Q.astype(np.float64),
                              with_stats=True, with_margins=True)
    ref = ref.reshape(-1)
    r = parity_bar.check(f"queries m={len(Q)} w={w_}", got, ref, mag, mg)
    print(f"  {parity_bar.fmt(r)}", flush=True)
    return ref


def test_sphere_inside_outside(dev, oracle_mod):
    import torch
    import paper_2405_16634_amd as w
    c = synth.fibonacci_sphere(2000, 0)
    ctx = w.Context(0)
    x, _ = ctx.normalize(torch.from_numpy(c.points).to(dev))
    ctx.build(x)
    xh = x.cpu().numpy().astype(np.float64)
    nrm = xh / np.linalg.norm(xh, axis=1, keepdims=True)
    r = np.linalg.norm(xh, axis=1).mean()
    mu = (nrm * (4.0 * np.pi * r * r / len(xh))).astype(np.float32)
    rng = np.random.default_rng(7)
    dirs = synth.random_unit(rng, 3000).astype(np.float64)
    rad = np.concatenate([rng.uniform(0.0, 0.7 * r, 1000), rng.uniform(1.3 * r, 2.5 * r, 1000),
                          rng.uniform(4.0, 9.0, 1000)])
    Q = (dirs * rad[:, None]).astype(np.float32)
    Q[0] = 0.0  # the centre
    got = ctx.winding_at(torch.from_numpy(mu).to(dev), 0.002,
                         torch.from_numpy(Q).to(dev)).cpu().numpy().astype(np.float64)
    _check(oracle_mod, xh, mu, Q, got, 0.002)
    # the treecode (c = 2) is within a few percent of the indicator
    assert np.all(np.abs(got[:1000] - 1.0) < 0.03)
    assert np.all(np.abs(got[1000:]) < 0.03)
    ctx.close()
    # exact sums (c large: nothing is accepted): F(0) = sum sigma / (4 pi r^2)
    # up to the jitter of the radii (Thm. 1)
    ctx = w.Context(0)
    ctx.build(x, c=1e6)
    f0 = ctx.winding_at(torch.from_numpy(mu).to(dev), 0.002,
                        torch.zeros(1, 3, device=dev)).cpu().numpy()[0]
    exact = float((4.0 * np.pi * r * r / len(xh)) / (4.0 * np.pi) * (1.0 / (xh ** 2).sum(1)).sum())
    assert f0 == pytest.approx(exact, rel=1e-5)
    assert f0 == pytest.approx(1.0, abs=3e-3)
    ctx.close()


@pytest.mark.parametrize("M", [1, 63, 1000, 20001])
def test_queries_match_the_oracle(dev, oracle_mod, M):
    import torch
    import paper_2405_16634_amd as w
    cloud = synth.torus_knot(20000, 5, with_init=False)
    ctx = w.Context(0)
    x, _ = ctx.normalize(torch.from_numpy(cloud.points).to(dev))
    ctx.build(x)
    xh = x.cpu().numpy()
    rng = np.random.default_rng(M)
    mu = (synth.random_unit(rng, cloud.n) * 1e-4).astype(np.float32)
    Q = rng.uniform(-1.2, 1.2, (M, 3)).astype(np.float32)
    if M > 100:
        Q[:50] = xh[rng.choice(cloud.n, 50, replace=False)]  # on points: the cutoff
        Q[50:60] = rng.uniform(-9.0, 9.0, (10, 3))            # far outside the root cell
    got = ctx.winding_at(torch.from_numpy(mu).to(dev), 0.002,
                         torch.from_numpy(Q).to(dev)).cpu().numpy().astype(np.float64)
    _check(oracle_mod, xh.astype(np.float64), mu, Q, got, 0.002)
    # the points themselves as queries give the winding number at the points
    if M == 1000:
        ctx.set_split(0)  # whole walks, as for queries: the same summation order
        at_pts = ctx.winding_at(torch.from_numpy(mu).to(dev), 0.002, x).cpu().numpy()
        direct = ctx.winding(torch.from_numpy(mu).to(dev), 0.002).cpu().numpy()
        assert np.array_equal(at_pts, direct)
    ctx.close()


def test_batched_tree_is_refused(dev):
    import torch
    import paper_2405_16634_amd as w
    pts = np.concatenate([synth.fibonacci_sphere(500, 0).points, synth.fibonacci_sphere(600, 1).points])
    off = np.array([0, 500, 1100], np.int64)
    ctx = w.Context(0)
    x, _ = ctx.normalize_batched(torch.from_numpy(pts).to(dev), off)
    ctx.build_batched(x, off)
    mu = torch.zeros(1100, 3, device=dev)
    with pytest.raises(w.WnncError):
        ctx.winding_at(mu, 0.002, torch.zeros(5, 3, device=dev))
    ctx.close()


def test_accept_test_is_strict_at_a_tie(dev, oracle_mod):
    """A query at exactly c 2^(1-d) from a node's x_B opens the node, on the
    device as in the oracle (dyadic coordinates: every distance is exact in
    FP32 too); one ulp farther, the representative is taken."""
    import torch
    import paper_2405_16634_amd as w
    print("[case] accept tie, two points, two queries", flush=True)
    x = np.array([[0.0625, 0.0625, 0.0625], [0.1875, 0.0625, 0.0625]], np.float32)
    mu = np.array([[0.01, 0.0, 0.0], [0.01, 0.0, 0.0]], np.float32)
    tie = np.array([0.625, 0.0625, 0.0625], np.float32)
    far = tie.copy()
    far[0] = np.nextafter(far[0], np.float32(1.0))
    Q = np.stack([tie, far])
    ctx = w.Context(0)
    ctx.build(torch.from_numpy(x).to(dev), 2.0, 15)
    ctx.set_flags(w.FLAG_COUNT_PAIRS)
    ctx.reset_stats()
    got = ctx.winding_at(torch.from_numpy(mu).to(dev), 1e-3, torch.from_numpy(Q).to(dev))
    torch.cuda.synchronize()
    pairs = ctx.stats()["pairs"][0]
    ctx.set_flags(0)
    ref, _, opairs = oracle_mod.Tree(x.astype(np.float64)).apply(
        "A", mu.astype(np.float64), 1e-3, 2.0, targets=Q.astype(np.float64), with_stats=True)
    assert list(opairs) == [2, 1] and pairs == 3
    assert np.allclose(got.cpu().numpy(), ref, rtol=1e-5, atol=0)
    ctx.close()
