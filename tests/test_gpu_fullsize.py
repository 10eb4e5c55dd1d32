"""Full-size checks on the benchmark workload (500k-point torus knot with
outliers, c = 2, D = 15, widths 0.002/0.016), in the launch configuration
bench.py times.

* Each operator over all points, compared with the FP64 oracle treecode on a
  seeded sample of targets (the oracle evaluates them one by one against the
  full tree), at the operator bar of `parity_bar.check`.
* The 40-iteration orientation: reproducibility, finite energies, its
  agreement with the generator's ground-truth normals, and, end to end,
  with the FP64 oracle's 40-iteration treecode run on the same cloud (flip
  rate <= 0.1 %; tests/golden/knot500k_orient_oracle.npz, written by
  make_knot500k_orient.py from the oracle alone).
* The 50k noisy ellipsoid union end to end against the oracle's 40-iteration
  run (flip rate), and the 2k sphere with exact sums (c huge) against the
  oracle's direct-sum run.
"""
import hashlib
import os

import numpy as np
import pytest

import parity_bar
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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
            assert np.all(np.isfinite(got))
            ref, mag, _, mg = T.apply(op, nu.astype(np.float64), w_, 2.0, targets=x[sample],
                                      with_stats=True, with_margins=True)
            r = parity_bar.check(f"fullsize {op} w={w_}", got[sample], sign * ref, mag, mg)
            print(f"  {op}: {parity_bar.fmt(r)}", flush=True)


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


def test_fullsize_orient_matches_oracle_run(knot):
    """The benchmark configuration end to end: the device's 40 iterations of
    Alg. 3 (in the tile, split and prefetch settings the autotuner picks, as
    the benchmark runs them) against the oracle's FP64 treecode run."""
    import torch
    ctx, cloud = knot["ctx"], knot["cloud"]
    g = np.load(os.path.join(GOLDEN, "knot500k_orient_oracle.npz"), allow_pickle=False)
    sha = hashlib.sha256(np.ascontiguousarray(cloud.points, np.float32).tobytes()).hexdigest()
    assert str(g["points_sha256"]) == sha, "the knot generator changed: rerun the script"
    print("[case] fullsize orient vs oracle (autotuned launch settings)", flush=True)
    ctx.autotune()
    mu = ctx.orient(40, 0.002, 0.016)
    E = np.array(ctx.energy(40))
    nrm = ctx.normals(mu).cpu().numpy().astype(np.float64)
    n_o = g["n16"].astype(np.float64) / 32767.0
    dots = (nrm * n_o).sum(1)
    flip = float((dots <= 0).mean())
    ang = np.degrees(np.arccos(np.clip(dots, -1, 1)))
    erel = np.abs(E - g["E"]) / g["E"]
    surf = np.isfinite(cloud.normals).all(axis=1)
    print(f"  flip={flip:.2e} (surface {(dots[surf] <= 0).mean():.2e}, outliers "
          f"{(dots[~surf] <= 0).mean():.2e}) median angle {np.median(ang):.2e} deg; "
          f"energy rel diff max {erel.max():.2e} (E40 {E[-1]:.4e} vs {g['E'][-1]:.4e})", flush=True)
    assert flip <= 1e-3
    assert E[0] == g["E"][0]
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
