"""Split walks combined inside the moment pass.

In Alg. 3's iterations, the combining pass of a split walk (the parts' sums
added in part order, then the walk's epilogue) runs inside the moment pass
that reads the walk's output when the 64-target groups line up with that
pass's wavefronts (every cloud starting at a multiple of 64 points).  It is
the same arithmetic in the same order as the separate combining launch, so
the orientation, the per-iteration energies (the step length's reductions)
and the pair counts are identical bit for bit to a run with
WNNC_FLAG_SEPARATE_COMBINE; a forest whose clouds do not line up takes the
separate launches either way.
"""
import numpy as np
import pytest

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


def _run(w, ctx, flags, iters):
    ctx.set_flags(flags)
    mu = ctx.orient(iters, 0.002, 0.016).clone()
    e = np.asarray(ctx.energy(iters)).copy()
    ctx.set_flags(flags | w.FLAG_COUNT_PAIRS)
    ctx.reset_stats()
    mu2 = ctx.orient(iters, 0.002, 0.016).clone()
    pairs = list(ctx.stats()["pairs"][:3])
    ctx.set_flags(0)
    return mu, e, mu2, pairs


@pytest.mark.parametrize("case", ["knot20k_split64", "union3077_split128", "aligned_forest",
                                  "ragged_forest"])
def test_fused_combining_is_bit_identical(dev, case):
    import paper_2405_16634_amd as w
    print(f"[case] fused combine {case}", flush=True)
    ctx = w.Context(0)
    if case.endswith("forest"):
        # clouds starting at multiples of 64 points line up with the moment
        # pass; a second cloud starting at point 3077 does not
        knot = synth.torus_knot(12800, 5, with_init=False).points
        if case == "aligned_forest":
            clouds = [knot, synth.ellipsoid_union(4096, 9, noise=0.001, with_init=False).points]
        else:
            clouds = [synth.ellipsoid_union(3077, 9, noise=0.001, with_init=False).points, knot]
        off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])]).astype(np.int64)
        x, _ = ctx.normalize_batched(_t(np.concatenate(clouds), dev), off)
        ctx.build_batched(x, off)
        split = 64
    else:
        cloud = (synth.torus_knot(20000, 5, with_init=False) if case.startswith("knot")
                 else synth.ellipsoid_union(3077, 9, noise=0.001, with_init=False))
        x, _ = ctx.normalize(_t(cloud.points, dev))
        ctx.build(x)
        split = int(case.rsplit("split", 1)[1])
    ctx.set_tile(1)
    ctx.set_split(split)
    iters = 6
    fused = _run(w, ctx, 0, iters)
    separate = _run(w, ctx, w.FLAG_SEPARATE_COMBINE, iters)
    for a, b in ((fused[0], separate[0]), (fused[2], separate[2])):
        assert bool((a == b).all()), case
    assert np.array_equal(fused[1], separate[1]), case
    assert fused[3] == separate[3], case
    # reproducible bit for bit
    again = _run(w, ctx, 0, iters)
    assert bool((again[0] == fused[0]).all())
    assert np.isfinite(fused[0].cpu().numpy()).all()
    ctx.close()


def test_unknown_flags_are_rejected(dev):
    import paper_2405_16634_amd as w
    ctx = w.Context(0)
    with pytest.raises(Exception):
        ctx.set_flags(1 << 12)
    ctx.set_flags(w.FLAG_SEPARATE_COMBINE)
    ctx.set_flags(0)
    ctx.close()
