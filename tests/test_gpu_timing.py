"""Per-launch timing (WNNC_FLAG_TIME_KERNELS, WNNC_FLAG_TIME_TRAVERSAL): the
events ride on the kernels' own dispatches.  Timing changes no result,
every timed kind gets a positive time, and the timed kernels fit inside the
wall time of the run."""
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_timed_run_is_identical_and_consistent():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_16634_amd as w
    w.load_library()
    dev = torch.device("cuda:0")
    cloud = synth.torus_knot(20000, 5, with_init=False)
    print("[case] timed orient knot20k", flush=True)
    stream = torch.cuda.current_stream()
    ctx = w.Context(0, stream)
    x, _ = ctx.normalize(torch.from_numpy(cloud.points).to(dev))
    ctx.build(x, 2.0, 15)
    mu0 = ctx.orient(40, 0.002, 0.016).clone()
    ctx.set_flags(w.FLAG_TIME_KERNELS)
    ctx.reset_stats()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    mu1 = ctx.orient(40, 0.002, 0.016).clone()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = e0.elapsed_time(e1)
    st = ctx.stats()
    ctx.set_flags(0)
    assert bool((mu0 == mu1).all())
    calls = st["calls"]
    assert calls[0] == 79 and calls[1] == 40 and calls[2] == 40
    for k in range(3):
        assert st["traverse_ms"][k] > 0
    assert st["moments_ms"] > 0 and st["combine_ms"] >= 0
    timed = sum(st["traverse_ms"][:3]) + st["moments_ms"] + st["combine_ms"]
    print(f"  wall {wall:.3f} ms, timed kernels {timed:.3f} ms", flush=True)
    assert timed <= wall * 1.001 + 0.01
    assert timed >= 0.5 * wall
    # traversal launches only: the same traversal times, no moment time
    ctx.set_flags(w.FLAG_TIME_TRAVERSAL)
    ctx.reset_stats()
    mu3 = ctx.orient(40, 0.002, 0.016).clone()
    torch.cuda.synchronize()
    st3 = ctx.stats()
    ctx.set_flags(0)
    assert bool((mu0 == mu3).all())
    assert st3["moments_ms"] == 0 and st3["combine_ms"] == 0
    for k in range(3):
        assert st3["traverse_ms"][k] > 0
        assert abs(st3["traverse_ms"][k] - st["traverse_ms"][k]) <= 0.2 * st["traverse_ms"][k]
    with pytest.raises(w.WnncError):
        ctx.set_flags(1 << 12)
    # the untimed run after it gives the same result again
    mu2 = ctx.orient(40, 0.002, 0.016)
    assert bool((mu0 == mu2).all())
    ctx.close()
