"""Deferred subtrees in the traversal (wnnc_set_defer): a subtree that few
targets of a 64-target group need is walked afterwards by those targets
alone, packed across the lanes.  Every target makes the same Alg. 4
decisions and adds the same terms as in the lockstep walk, so:

* pair counts are identical for every deferral threshold, on a single cloud,
  with split walks, with leaves of several points and on a batched forest;
* outputs agree with the lockstep walk at the summation-order bound of
  `parity_bar.same_terms` (the deferred steps add each term to the FP64 sum
  at once, the lockstep walk through FP32 running sums of a few terms), and
  Alg. 3 gives the same orientation (no flips);
* runs are reproducible bit for bit (the packed walks and the sums into the
  targets run in a fixed order);
* the result matches the oracle at the operator bar (`parity_bar.check`).
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


def _mags(oracle_mod, x, off, mu, rho, w=0.002):
    """Per target, the oracle's sum of term magnitudes of A, G and A^T, cloud
    by cloud (each cloud of a batch has its own tree)."""
    xs = x.cpu().numpy().astype(np.float64)
    mus = mu.cpu().numpy().astype(np.float64)
    rhos = rho.cpu().numpy().astype(np.float64)
    mags = [[], [], []]
    for c in range(len(off) - 1):
        sl = slice(int(off[c]), int(off[c + 1]))
        T = oracle_mod.Tree(xs[sl])
        for k, (op, nu) in enumerate((("A", mus[sl]), ("G", mus[sl]), ("AT", rhos[sl]))):
            _, mag, _ = T.apply(op, nu, w, 2.0, with_stats=True)
            mags[k].append(mag)
    return [np.concatenate(m) for m in mags]


def _ops(w, ctx, mu, rho):
    ctx.set_flags(w.FLAG_COUNT_PAIRS)
    ctx.reset_stats()
    out = (ctx.winding(mu, 0.002).clone(), ctx.gradient(mu, 0.002).clone(),
           ctx.adjoint(rho, 0.002).clone())
    pairs = list(ctx.stats()["pairs"][:3])
    ctx.set_flags(0)
    return out, pairs


@pytest.mark.parametrize("case", ["knot20k", "knot20k_leafcap8", "batched"])
def test_deferral_changes_only_the_summation_order(dev, oracle_mod, case):
    import paper_2405_16634_amd as w
    print(f"[case] deferral {case}", flush=True)
    ctx = w.Context(0)
    if case == "batched":
        clouds = [synth.torus_knot(20000, 5, with_init=False).points,
                  synth.ellipsoid_union(3077, 9, noise=0.001, with_init=False).points,
                  np.repeat(np.random.default_rng(3).uniform(-1, 1, (4, 3)).astype(np.float32), 3, 0)]
        off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])]).astype(np.int64)
        x, _ = ctx.normalize_batched(_t(np.concatenate(clouds), dev), off)
        ctx.build_batched(x, off)
        n = int(off[-1])
        leaf_cap = 1
    else:
        cloud = synth.torus_knot(20000, 5, with_init=False)
        x, _ = ctx.normalize(_t(cloud.points, dev))
        leaf_cap = 8 if case.endswith("leafcap8") else 1
        ctx.build(x, 2.0, 15, leaf_cap)
        n = cloud.n
        off = np.array([0, n], np.int64)
    rng = np.random.default_rng(21)
    mu = _t(synth.random_unit(rng, n) * 1e-4, dev)
    rho = _t(rng.standard_normal(n), dev)
    if leaf_cap == 1:
        mags = _mags(oracle_mod, x, off, mu, rho)
    else:  # the oracle's tree with the same leaf capacity
        xs = x.cpu().numpy().astype(np.float64)
        T = oracle_mod.Tree(xs, 15, leaf_cap)
        mags = [T.apply(op, nu.cpu().numpy().astype(np.float64), 0.002, 2.0, with_stats=True)[1]
                for op, nu in (("A", mu), ("G", mu), ("AT", rho))]
    ctx.set_tile(1)
    ctx.set_prefetch(False)
    res = {}
    for split in (0, 64):
        ctx.set_split(split)
        for k in (0, 1, 8, 32, 64):
            ctx.set_defer(k)
            assert ctx.defer() == k
            out, pairs = _ops(w, ctx, mu, rho)
            o5 = ctx.orient(5, 0.002, 0.016).clone()
            res[(split, k)] = (out, pairs, o5)
    ref_out, ref_pairs, ref_o5 = res[(0, 0)]
    worst = 0.0
    for key, (out, pairs, o5) in res.items():
        assert pairs == ref_pairs, key
        for op, a, b, mag in zip(("A", "G", "AT"), out, ref_out, mags):
            worst = max(worst, parity_bar.same_terms(f"{case} {key} {op}", a.cpu().numpy(),
                                                     b.cpu().numpy(), mag))
        assert ((o5 * ref_o5).sum(1) <= 0).float().mean().item() == 0.0, key
    print(f"  {case}: largest summation-order difference {worst:.2e} M", flush=True)
    # reproducible bit for bit
    ctx.set_split(64)
    ctx.set_defer(32)
    again, _ = _ops(w, ctx, mu, rho)
    for a, b in zip(again, res[(64, 32)][0]):
        assert bool((a == b).all())
    ctx.close()


def test_deferred_walk_matches_oracle(dev, oracle_mod):
    """The deferred walk (every subtree of at most 64 lanes, i.e. nearly all
    of the walk below the root region) against the oracle's treecode."""
    import paper_2405_16634_amd as w
    import oracle
    cloud = synth.ellipsoid_union(3077, 9, noise=0.001, with_init=False)
    print("[case] deferral 64 ragged3077 vs oracle", flush=True)
    ctx = w.Context(0)
    x, _ = ctx.normalize(_t(cloud.points, dev))
    x_or, _, sc = oracle.normalize(cloud.points)
    ctx.build(x)
    ctx.set_defer(64)
    T = oracle_mod.Tree(x_or)
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
            r = parity_bar.check(f"defer 64 {op} w={w_}", got[op], ref, mag, mg)
            print(f"  {op} w={w_}: {parity_bar.fmt(r)}", flush=True)
    ctx.close()


def test_defer_setting_is_checked(dev):
    import paper_2405_16634_amd as w
    ctx = w.Context(0)
    assert ctx.defer() == 32
    for bad in (-1, 65):
        with pytest.raises(w.WnncError):
            ctx.set_defer(bad)
    ctx.close()
