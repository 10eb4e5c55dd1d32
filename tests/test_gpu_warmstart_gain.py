"""What the trained warm-start network gains over the method without it.

Held-out clouds (seeds not used in training): a torus knot with 2 %
outliers and a noise-free ellipsoid union.  The plain method (40 iterations
from mu = 0) is the reference.  Equal accuracy, on the surface points (outliers
have no normal): the warm-started result disagrees with the plain one on at
most 0.1 % of them, and orients at least as many correctly against the
generator's normals (P_co within 0.1 %), while running fewer iterations and
less wall time.  The trained network's raw predictions must be far closer to
the plain normals than an untrained network's, and an untrained network must
end in correct normals through the self-check fallback.

What the network adds: the same short schedule (6 iterations, widths
0.016 -> 0.002) started from mu = 0 instead of the network's prediction
misses equal accuracy on both clouds.  Also run: the warm start continued
at the final width until at most 0.1 % of the points change sign per WNNC
update, or the count stops falling (at most 40 iterations), and the plain
method from random initial vectors scaled by the mean area (reported).
"""
import os
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2405_16634_amd", "data", "warmstart_mlp.npy")


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_16634_amd as w
    w.load_library()
    return torch.device("cuda:0")


def _flip(a, b, mask=None):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    ok = (np.linalg.norm(a, axis=1) > 0) & (np.linalg.norm(b, axis=1) > 0)
    if mask is not None:
        ok &= mask
    return float(((a[ok] * b[ok]).sum(1) <= 0).mean())


def _run(dev, cloud, params, controls=False):
    import torch
    import paper_2405_16634_amd as w
    ctx = w.Context(0)
    x, norm = ctx.normalize(torch.from_numpy(cloud.points).to(dev))
    ctx.build(x)
    ctx.orient(40)  # warm caches and code paths once
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mu_p = ctx.orient(40)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    mu_w, rep = ctx.warm_orient(params)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    pred = torch.empty_like(mu_p)
    w.wnnc_mlp_forward(ctx.handle, params, ctx.features(), pred)
    torch.cuda.synchronize()
    out = dict(plain=mu_p.cpu().numpy(), warm=mu_w.cpu().numpy(), pred=pred.cpu().numpy(),
               t_plain=t_plain, t_warm=t_warm, rep=rep)
    if controls:
        out["short"] = ctx.orient(6, 0.002, 0.016).cpu().numpy()
        conv, rep_c = ctx.warm_orient(params, max_iters=40, stop_frac=1e-3)
        out["conv"], out["rep_conv"] = conv.cpu().numpy(), rep_c
        sig = cloud.area * norm.scale ** 2 / cloud.n
        m0 = torch.from_numpy((cloud.mu0.astype(np.float64) * sig).astype(np.float32)).to(dev)
        out["random"] = ctx.orient(40, mu0=m0).cpu().numpy()
    ctx.close()
    return out


@pytest.mark.parametrize("name", ["knot100k", "ellipsoids60k"])
def test_trained_warm_start_gains(dev, name):
    import torch
    from paper_2405_16634_amd import warmstart as ws
    if not os.path.exists(WEIGHTS):
        pytest.fail(f"trained weights missing: {WEIGHTS}")
    params = ws.load_params(WEIGHTS)
    cloud = (synth.torus_knot(100000, 777) if name == "knot100k"
             else synth.ellipsoid_union(60000, 555, noise=0.0))
    gt = cloud.normals.astype(np.float64)
    surf = np.isfinite(gt).all(axis=1)
    r = _run(dev, cloud, params, controls=True)
    flip_warm = _flip(r["warm"], r["plain"], surf)
    flip_short = _flip(r["short"], r["plain"], surf)
    flip_conv = _flip(r["conv"], r["plain"], surf)
    flip_rand = _flip(r["random"], r["plain"], surf)
    pco_short = 1.0 - _flip(r["short"], gt, surf)
    pco_rand = 1.0 - _flip(r["random"], gt, surf)
    flip_pred = _flip(r["pred"], r["plain"], surf)
    pco_plain = 1.0 - _flip(r["plain"], gt, surf)
    pco_warm = 1.0 - _flip(r["warm"], gt, surf)
    untrained = torch.from_numpy(ws.init_params(123)).to(dev)
    ru = _run(dev, cloud, untrained)
    flip_pred_u = _flip(ru["pred"], ru["plain"], surf)
    print(f"  {name}: warm flip={flip_warm:.2e} (all points {_flip(r['warm'], r['plain']):.2e}) "
          f"P_co plain={pco_plain:.5f} warm={pco_warm:.5f} iters={r['rep']['iterations']} "
          f"fallback={r['rep']['fallback']} t_plain={r['t_plain']*1e3:.1f} ms "
          f"t_warm={r['t_warm']*1e3:.1f} ms pred flip trained={flip_pred:.3f} "
          f"untrained={flip_pred_u:.3f} untrained_fallback={ru['rep']['fallback']} "
          f"(last-update disagree {ru['rep']['max_disagree']:.2e}, prediction disagree "
          f"{ru['rep']['max_pred_disagree']:.3f})", flush=True)
    print(f"  {name}: no-network control (6 iterations from mu = 0): flip={flip_short:.2e} "
          f"P_co={pco_short:.5f}; until convergence: iters={r['rep_conv']['iterations']} "
          f"flip={flip_conv:.2e}; random-init plain: flip={flip_rand:.2e} P_co={pco_rand:.5f}",
          flush=True)
    # what the network adds: the same short schedule without it misses
    # equal accuracy, with it the result meets it
    assert flip_short > 1e-3
    assert flip_warm <= 1e-3
    # run until the sign changes stop: still equal accuracy, within the cap
    assert flip_conv <= 1e-3 and not r["rep_conv"]["fallback"]
    assert r["rep"]["iterations"] <= r["rep_conv"]["iterations"] <= 40
    # the trained predictions orient most points already; an untrained net does not
    assert flip_pred < 0.5 * flip_pred_u
    # equal accuracy, fewer iterations, less time
    assert flip_warm <= 1e-3
    assert pco_warm >= pco_plain - 1e-3
    assert not r["rep"]["fallback"]
    assert r["rep"]["iterations"] < 40
    assert r["t_warm"] < r["t_plain"]
    # an untrained network's prediction carries no information: the self
    # check sees it and the plain method reruns, ending correct
    assert ru["rep"]["fallback"]
    assert ru["rep"]["max_pred_disagree"] > 0.4
    assert ru["rep"]["iterations"] == 6 + 40
    assert _flip(ru["warm"], ru["plain"], surf) <= 1e-3
