"""Batched clouds (one forest, one launch per operator) and traversal tile
shapes.

* every cloud of a batch has the octree its standalone build has (node sets
  against the oracle's recursive partition of that cloud alone);
* operators on a batch equal the oracle treecode of each cloud alone (the
  operator bar of `parity_bar.check`);
* the 40-iteration orientation of a batch agrees with running each cloud
  alone (per-cloud step lengths and energies);
* the tile shape (targets per lane) and split walks change neither a
  decision nor a pair count, only where the walk's FP32 running sums are
  added to its FP64 sums (results agree at the summation-order bound of
  `parity_bar.same_terms`); the prefetching walk, which visits the same
  nodes in the same order, changes no result bit;
* walks split into node-range parts make the same decisions as whole walks;
* the 64-cloud workload (sizes log-uniform in [5k, 200k]) batched against
  the clouds one by one.
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


def _batch():
    rng = np.random.default_rng(40)
    clouds = [
        synth.ellipsoid_union(3077, 9, noise=0.001, with_init=False).points,
        rng.uniform(-1, 1, (1, 3)).astype(np.float32),
        np.repeat(rng.uniform(-1, 1, (3, 3)).astype(np.float32), 3, axis=0),
        synth.fibonacci_sphere(2000, 0).points,
        synth.torus_knot(20000, 5, with_init=False).points,
        rng.uniform(-1, 1, (300, 3)).astype(np.float32),
    ]
    off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])]).astype(np.int64)
    return clouds, off


def _sets(depth, begin, end, order, lo=0):
    return {(int(d), tuple(sorted((order[b:e] - lo).tolist()))) for d, b, e in zip(depth, begin, end)}


def test_batched_normalize_and_forest(dev, oracle_mod):
    import torch
    import paper_2405_16634_amd as w
    clouds, off = _batch()
    P = torch.from_numpy(np.concatenate(clouds)).to(dev)
    ctx = w.Context(0)
    x, norms = ctx.normalize_batched(P, off)
    ctx.build_batched(x, off)
    st = ctx.stats()
    assert st["n_clouds"] == len(clouds)
    xh = x.cpu().numpy()
    d, leaf, b, e, perm = ctx.tree()
    total = 0
    for k, c in enumerate(clouds):
        xo, _, sc = oracle_mod.normalize(c)
        assert np.array_equal(xh[off[k]:off[k + 1]], xo)
        assert norms[k].scale == pytest.approx(sc, rel=1e-15)
        # nodes of cloud k: those whose points lie in its caller range
        sel = (perm[b] >= off[k]) & (perm[b] < off[k + 1])
        T = oracle_mod.Tree(xo.astype(np.float64))
        od, ol, obg, oen, oo = T.export()
        assert _sets(d[sel], b[sel], e[sel], perm, off[k]) == _sets(od, obg, oen, oo)
        total += int(sel.sum())
    assert total == len(d)
    ctx.close()


@pytest.mark.parametrize("split", [0, 48])
def test_batched_operators(dev, oracle_mod, split):
    """Every cloud against the oracle; with split = 48 the walks run as many
    short parts that start deep in the tree."""
    import torch
    import paper_2405_16634_amd as w
    clouds, off = _batch()
    P = torch.from_numpy(np.concatenate(clouds)).to(dev)
    ctx = w.Context(0)
    x, _ = ctx.normalize_batched(P, off)
    ctx.build_batched(x, off)
    ctx.set_split(split)
    st = ctx.stats()
    assert (st["n_tasks"] > st["n_groups"]) == (split > 0)
    xh = x.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(5)
    n = int(off[-1])
    mu = (synth.random_unit(rng, n) * 1e-4).astype(np.float32)
    rho = rng.standard_normal(n).astype(np.float32)
    for w_ in (0.002, 0.016):
        s = ctx.winding(torch.from_numpy(mu).to(dev), w_).cpu().numpy()
        g = ctx.gradient(torch.from_numpy(mu).to(dev), w_).cpu().numpy()
        at = ctx.adjoint(torch.from_numpy(rho).to(dev), w_).cpu().numpy()
        for k in range(len(clouds)):
            a, b_ = off[k], off[k + 1]
            T = oracle_mod.Tree(xh[a:b_])
            for op, got, nu, sign in (("A", s, mu, 1.0), ("G", g, mu, -1.0), ("AT", at, rho, 1.0)):
                ref, mag, _, mg = T.apply(op, nu[a:b_].astype(np.float64), w_, 2.0,
                                          with_stats=True, with_margins=True)
                parity_bar.check(f"split={split} cloud {k} {op} w={w_}", got[a:b_], sign * ref,
                                 mag, mg)
    ctx.close()


def test_batched_orient_equals_single(dev):
    import torch
    import paper_2405_16634_amd as w
    clouds, off = _batch()
    P = torch.from_numpy(np.concatenate(clouds)).to(dev)
    ctx = w.Context(0)
    x, _ = ctx.normalize_batched(P, off)
    ctx.build_batched(x, off)
    mu_b = ctx.orient(40, 0.002, 0.016).cpu().numpy()
    E_b = np.array(ctx.energy(40))  # (40, clouds)
    ctx.close()
    for k, c in enumerate(clouds):
        ctx = w.Context(0)
        xk, _ = ctx.normalize(torch.from_numpy(c).to(dev))
        ctx.build(xk)
        mu_s = ctx.orient(40, 0.002, 0.016).cpu().numpy()
        E_s = np.array(ctx.energy(40))
        ctx.close()
        mb = mu_b[off[k]:off[k + 1]]
        nz = np.linalg.norm(mu_s, axis=1) > 0
        flip = ((mb[nz] * mu_s[nz]).sum(1) <= 0).mean() if nz.any() else 0.0
        print(f"  cloud {k} n={len(c)} flip={flip:.2e} E39 batch={E_b[-1, k]:.6e} single={E_s[-1]:.6e}",
              flush=True)
        assert flip <= 1e-3
        assert E_b[0, k] == pytest.approx(0.25 * len(c))
        assert np.allclose(E_b[:, k], E_s, rtol=1e-3, atol=1e-9)


def _mags(oracle_mod, x, mu, rho=None, w=0.002):
    """The oracle's per-target sums of term magnitudes for A, G (and A^T)."""
    T = oracle_mod.Tree(x.cpu().numpy().astype(np.float64))
    out = []
    for op, nu in (("A", mu), ("G", mu)) + ((("AT", rho),) if rho is not None else ()):
        _, mag, _ = T.apply(op, nu.cpu().numpy().astype(np.float64), w, 2.0, with_stats=True)
        out.append(mag)
    return out


def _same_orientation(a, b, label):
    a = a.cpu().numpy().astype(np.float64)
    b = b.cpu().numpy().astype(np.float64)
    flip = float(((a * b).sum(1) <= 0).mean())
    rel = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    print(f"  {label}: five iterations flip={flip:.1e} rel={rel:.2e}", flush=True)
    assert flip == 0.0 and rel <= 1e-5, label


def test_tile_shapes_change_only_the_summation_grouping(dev, oracle_mod):
    """Tile shapes 1, 2, 4 with and without prefetch: equal pair counts;
    bit-identical with and without prefetch (the same visits in the same
    order); across shapes within the summation-order bound, and five
    iterations of Alg. 3 agree."""
    import torch
    import paper_2405_16634_amd as w
    cloud = synth.torus_knot(20000, 5, with_init=False)
    ctx = w.Context(0)
    x, _ = ctx.normalize(torch.from_numpy(cloud.points).to(dev))
    ctx.build(x)
    rng = np.random.default_rng(2)
    mu = torch.from_numpy((synth.random_unit(rng, cloud.n) * 1e-4).astype(np.float32)).to(dev)
    magA, magG = _mags(oracle_mod, x, mu)
    ctx.set_split(0)  # whole walks
    ctx.set_defer(0)  # every subtree in lockstep
    ref = ref_pairs = None
    for tpl in (1, 2, 4):
        per = {}
        for pf in (False, True):
            ctx.set_tile(tpl)
            ctx.set_prefetch(pf)
            assert ctx.tile() == tpl and ctx.prefetch() == pf
            per[pf] = (ctx.winding(mu, 0.002).clone(), ctx.gradient(mu, 0.002).clone(),
                       ctx.orient(5, 0.002, 0.016).clone())
            ctx.set_flags(w.FLAG_COUNT_PAIRS)
            ctx.reset_stats()
            ctx.winding(mu, 0.002)
            ctx.gradient(mu, 0.002)
            pairs = list(ctx.stats()["pairs"][:3])
            ctx.set_flags(0)
            if ref_pairs is None:
                ref_pairs = pairs
            assert pairs == ref_pairs, (tpl, pf)
        for a, b in zip(per[False], per[True]):
            assert bool((a == b).all()), tpl
        out = per[False]
        if ref is None:
            ref = out
            continue
        ra = parity_bar.same_terms(f"tpl={tpl} A", out[0].cpu().numpy(), ref[0].cpu().numpy(), magA)
        rg = parity_bar.same_terms(f"tpl={tpl} G", out[1].cpu().numpy(), ref[1].cpu().numpy(), magG)
        print(f"  tpl={tpl}: A {ra:.2e} M, G {rg:.2e} M", flush=True)
        _same_orientation(out[2], ref[2], f"tpl={tpl}")
    ctx.close()


def test_split_walks_make_the_same_decisions(dev, oracle_mod):
    """Walks split into node-range parts (down to 32 visits, so that parts
    start deep in the tree and rebuild long ancestor chains) count exactly
    the pairs of whole walks, agree with them at the summation-order bound,
    and are bit-identical across prefetch settings."""
    import torch
    import paper_2405_16634_amd as w
    cloud = synth.torus_knot(20000, 5, with_init=False)
    ctx = w.Context(0)
    x, _ = ctx.normalize(torch.from_numpy(cloud.points).to(dev))
    ctx.build(x)
    ngroups = (cloud.n + 63) // 64
    rng = np.random.default_rng(2)
    mu = torch.from_numpy((synth.random_unit(rng, cloud.n) * 1e-4).astype(np.float32)).to(dev)
    rho = torch.from_numpy(rng.standard_normal(cloud.n).astype(np.float32)).to(dev)
    mags = _mags(oracle_mod, x, mu, rho)
    res = {}
    ctx.set_defer(0)  # the lockstep walk in both prefetch settings
    for split in (0, 32, 256):
        for pf in (False, True):
            ctx.set_tile(1)
            ctx.set_split(split)
            ctx.set_prefetch(pf)
            assert ctx.split() == split
            ctx.set_flags(w.FLAG_COUNT_PAIRS)
            ctx.reset_stats()
            out = (ctx.winding(mu, 0.002).clone(), ctx.gradient(mu, 0.002).clone(),
                   ctx.adjoint(rho, 0.002).clone())
            st = ctx.stats()
            ctx.set_flags(0)
            assert st["n_groups"] == ngroups
            if split == 0:
                assert st["n_tasks"] == ngroups
            else:
                assert st["n_tasks"] > ngroups, (split, st["n_tasks"])
            o5 = ctx.orient(5, 0.002, 0.016).clone()
            res[(split, pf)] = (out, list(st["pairs"]), o5)
            print(f"  split={split} pf={int(pf)} tasks={st['n_tasks']} pairs={st['pairs']}", flush=True)
    ref_out, ref_pairs, ref_o5 = res[(0, False)]
    for (split, pf), (out, pairs, o5) in res.items():
        assert pairs == ref_pairs, (split, pf)
        other = res[(split, not pf)]
        for a, b in zip(out, other[0]):
            assert bool((a == b).all()), (split, pf)
        for op, a, b, mag in zip(("A", "G", "AT"), out, ref_out, mags):
            parity_bar.same_terms(f"split={split} pf={int(pf)} {op}", a.cpu().numpy(),
                                  b.cpu().numpy(), mag)
        _same_orientation(o5, ref_o5, f"split={split} pf={int(pf)}")
    ctx.close()


def test_autotune_keeps_the_fastest(dev):
    import torch
    import paper_2405_16634_amd as w
    cloud = synth.torus_knot(20000, 5, with_init=False)
    ctx = w.Context(0)
    x, _ = ctx.normalize(torch.from_numpy(cloud.points).to(dev))
    ctx.build(x)
    ms = ctx.autotune(0.002)
    assert len(ms) == w.AUTOTUNE_CONFIGS and all(v > 0 for v in ms.values())
    assert {k[:2] for k in ms} == {(t, p) for t in (1, 2, 4) for p in (0, 1)}
    # the fastest, except that a setting later in the list must beat the
    # best so far by more than 1 %
    best = None
    for key, t in ms.items():
        if best is None or t < ms[best] * 0.99:
            best = key
    assert (ctx.tile(), int(ctx.prefetch()), ctx.split()) == best
    assert 0.99 * ms[best] <= min(ms.values())
    # per operator kind the walk may differ from the chosen one; the
    # position-gradient kinds, which the tuning iterations do not run,
    # follow it
    po = ctx.stats()["prefetch_ops"]
    assert 0 <= po < 32
    for k in (3, 4):
        assert (po >> k) & 1 == int(ctx.prefetch())
    ctx.set_prefetch(False)
    assert ctx.stats()["prefetch_ops"] == 0
    ctx.set_prefetch(True)
    assert ctx.stats()["prefetch_ops"] == 31
    ctx.close()


def test_batched64_workload_matches_one_by_one(dev):
    """The 64-cloud workload: sizes floor(exp(U[ln 5e3, ln 2e5])) (seed 1),
    noise-free ellipsoid unions; one forest, one launch per operator."""
    import torch
    import paper_2405_16634_amd as w
    sizes = synth.batched_sizes(64, 1)
    clouds = synth.batched_clouds(64, 1, sizes)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    print(f"[case] batched64 N={off[-1]}", flush=True)
    P = torch.from_numpy(np.concatenate([c.points for c in clouds])).to(dev)
    ctx = w.Context(0)
    x, _ = ctx.normalize_batched(P, off)
    ctx.build_batched(x, off)
    ctx.autotune(0.002)
    mu_b = ctx.orient(40, 0.002, 0.016).cpu().numpy()
    ctx.close()
    flips = []
    for k in range(0, 64, 9):
        ctx = w.Context(0)
        xk, _ = ctx.normalize(torch.from_numpy(clouds[k].points).to(dev))
        ctx.build(xk)
        mu_s = ctx.orient(40, 0.002, 0.016).cpu().numpy()
        ctx.close()
        flips.append(((mu_b[off[k]:off[k + 1]] * mu_s).sum(1) <= 0).mean())
    print(f"  flips one-by-one vs batched: max={max(flips):.2e}", flush=True)
    assert max(flips) <= 1e-3


def test_split_walks_with_zero_weight_regions(dev, oracle_mod):
    """Attributes zero on whole regions (zero-weight subtrees, which are not
    descended): parts that start below such ancestors must add nothing there.
    Split and whole walks against the oracle, and against each other."""
    import torch
    import paper_2405_16634_amd as w
    cloud = synth.torus_knot(20000, 11, with_init=False)
    ctx = w.Context(0)
    x, _ = ctx.normalize(torch.from_numpy(cloud.points).to(dev))
    ctx.build(x)
    xh = x.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(12)
    mu = (synth.random_unit(rng, cloud.n) * 1e-4).astype(np.float32)
    rho = rng.standard_normal(cloud.n).astype(np.float32)
    dead = xh[:, 0] > 0.1  # a slab of zero attributes
    mu[dead] = 0.0
    rho[dead] = 0.0
    T = oracle_mod.Tree(xh)
    outs = {}
    mags = {}
    for split in (0, 64):
        ctx.set_split(split)
        outs[split] = (ctx.winding(torch.from_numpy(mu).to(dev), 0.002).cpu().numpy(),
                       ctx.gradient(torch.from_numpy(mu).to(dev), 0.002).cpu().numpy(),
                       ctx.adjoint(torch.from_numpy(rho).to(dev), 0.002).cpu().numpy())
        for op, got, nu, sign in (("A", outs[split][0], mu, 1.0), ("G", outs[split][1], mu, -1.0),
                                  ("AT", outs[split][2], rho, 1.0)):
            ref, mag, _, mg = T.apply(op, nu.astype(np.float64), 0.002, 2.0, with_stats=True,
                                      with_margins=True)
            r = parity_bar.check(f"split={split} {op}", got, sign * ref, mag, mg)
            print(f"  split={split} {op}: {parity_bar.fmt(r)}", flush=True)
            mags[op] = mag
    for op, a, b in zip(("A", "G", "AT"), outs[0], outs[64]):
        parity_bar.same_terms(f"split 0 vs 64 {op}", a, b, mags[op])
    ctx.close()
