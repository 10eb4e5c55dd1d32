"""Full-size checks on the benchmark workload (500k-point torus knot with
outliers, c = 2, D = 15, widths 0.002/0.016), in the launch configuration
bench.py times.

* Each operator over all points, compared with the FP64 oracle treecode on a
  seeded sample of targets (the oracle evaluates them one by one against the
  full tree).
* The 40-iteration orientation: reproducibility, finite energies, and its
  agreement with the generator's ground-truth normals.
* The 50k noisy ellipsoid union end to end against the oracle's 40-iteration
  run (flip rate), and the 2k sphere with exact sums (c huge) against the
  oracle's direct-sum run.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def knot():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_2405_16634_amd as w
    cloud = synth.torus_knot(500000, 3)
    dev = torch.device("cuda:0")
    ctx = w.Context(0)
    x_dev, norm = ctx.normalize(torch.from_numpy(cloud.points).to(dev))
    ctx.build(x_dev)
    x_or, _, sc = oracle.normalize(cloud.points)
    assert np.array_equal(x_dev.cpu().numpy(), x_or)
    yield dict(ctx=ctx, cloud=cloud, x=x_or.astype(np.float64), sc=sc, dev=dev, norm=norm)
    ctx.close()


def test_fullsize_operators_on_sampled_targets(knot, oracle_mod):
    import torch
    ctx, cloud, x, sc, dev = knot["ctx"], knot["cloud"], knot["x"], knot["sc"], knot["dev"]
    n = cloud.n
    rng = np.random.default_rng(31)
    sig = cloud.area * sc * sc / n
    mu = (synth.random_unit(rng, n) * sig).astype(np.float32)
    rho = (0.5 - rng.uniform(0, 1, n)).astype(np.float32)
    sample = np.sort(rng.choice(n, 3000, replace=False))
    T = oracle_mod.Tree(x)
    for w_ in (0.002, 0.016):
        print(f"[case] fullsize ops w={w_}", flush=True)
        s = ctx.winding(torch.from_numpy(mu).to(dev), w_).cpu().numpy()
        g = ctx.gradient(torch.from_numpy(mu).to(dev), w_).cpu().numpy()
        at = ctx.adjoint(torch.from_numpy(rho).to(dev), w_).cpu().numpy()
        for op, got, nu, sign in (("A", s, mu, 1.0), ("G", g, mu, -1.0), ("AT", at, rho, 1.0)):
            ref, mag, _ = T.apply(op, nu.astype(np.float64), w_, 2.0, targets=x[sample], with_stats=True)
            assert np.all(np.isfinite(got[sample]))
            err = np.abs(got[sample] - sign * ref)
            if err.ndim == 2:
                err = np.linalg.norm(err, axis=1)
            frac = (err / mag > TOL).mean()
            print(f"  {op}: frac>tol={frac:.2e} max_rel={(err / mag).max():.2e}", flush=True)
            assert frac <= 2e-3


def test_fullsize_orient_properties(knot):
    import torch
    ctx, cloud, dev = knot["ctx"], knot["cloud"], knot["dev"]
    print("[case] fullsize orient", flush=True)
    mu1 = ctx.orient(40, 0.002, 0.016).clone()
    E = np.array(ctx.energy(40))
    mu2 = ctx.orient(40, 0.002, 0.016).clone()
    assert bool((mu1 == mu2).all())
    assert np.all(np.isfinite(E)) and E[0] == pytest.approx(0.25 * cloud.n)
    nrm = ctx.normals(mu1, knot["norm"].scale).cpu().numpy()
    ok = np.isfinite(cloud.normals).all(axis=1)
    dots = (nrm[ok] * cloud.normals[ok]).sum(1)
    pco = (dots > 0).mean()
    print(f"  P_co={pco:.5f} AE={((1 - dots) / 2).mean():.5f}", flush=True)
    assert pco > 0.99
    torch.cuda.synchronize()


def test_ellipsoids50k_orient_matches_oracle(oracle_mod):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_16634_amd as w
    cloud = synth.ellipsoid_union(50000, 2)
    print("[case] ellipsoids50k orient", flush=True)
    ctx = w.Context(0)
    x_dev, _ = ctx.normalize(torch.from_numpy(cloud.points).to("cuda:0"))
    ctx.build(x_dev)
    mu_g = ctx.orient(40, 0.02, 0.08).cpu().numpy().astype(np.float64)
    ctx.close()
    x_or, _, _ = oracle_mod.normalize(cloud.points)
    mu_o = oracle_mod.orient(x_or, iters=40, w1=0.02, w2=0.08, backend="tree")
    flip = ((mu_g * mu_o).sum(1) <= 0).mean()
    pco = ((mu_g * cloud.normals).sum(1) > 0).mean()
    print(f"  flip_vs_oracle={flip:.2e} P_co_gpu={pco:.5f}", flush=True)
    assert flip <= 1e-3


def test_sphere2k_exact_sums_match_oracle_direct(oracle_mod):
    """The 2k-sphere case with exact O(N^2) sums: a huge c makes the treecode
    open every node, and the oracle runs the direct sums."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_16634_amd as w
    cloud = synth.fibonacci_sphere(2000, 0)
    ctx = w.Context(0)
    x_dev, _ = ctx.normalize(torch.from_numpy(cloud.points).to("cuda:0"))
    ctx.build(x_dev, c=1e6)
    mu_g = ctx.orient(40, 0.002, 0.016).cpu().numpy().astype(np.float64)
    ctx.close()
    x_or, _, _ = oracle_mod.normalize(cloud.points)
    mu_o = oracle_mod.orient(x_or, iters=40, w1=0.002, w2=0.016, backend="direct")
    flip = ((mu_g * mu_o).sum(1) <= 0).mean()
    ng = mu_g / np.linalg.norm(mu_g, axis=1, keepdims=True)
    no = mu_o / np.linalg.norm(mu_o, axis=1, keepdims=True)
    ang = np.degrees(np.arccos(np.clip((ng * no).sum(1), -1, 1)))
    print(f"  flip={flip:.2e} mean_angle={ang.mean():.2e} deg", flush=True)
    assert flip == 0.0
    assert ang.max() < 0.05
