"""The no-allocation entry point (wnnc_winding_grad_x_noalloc) through the C
ABI: the same result as wnnc_winding_grad_x, bit for bit (the same kernels on
the same inputs), on two calls in a row, the second on a smaller cloud (the
static scratch keeps the first call's contents); sizes beyond its limit are
refused before any work; and no device allocation happens during the call
(torch's allocator is bypassed, so its counters cannot see the library:
the HIP-level free-memory figure is compared instead)."""
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


def _case(dev, cloud, seed, oracle_mod, with_oracle):
    import torch
    import paper_2405_16634_amd as w
    import oracle
    ctx = w.Context(0)
    x, _ = ctx.normalize(torch.from_numpy(cloud.points).to(dev))
    ctx.build(x)
    rng = np.random.default_rng(seed)
    x_or, _, sc = oracle.normalize(cloud.points)
    mu = (synth.random_unit(rng, cloud.n) * (cloud.area * sc * sc / cloud.n)).astype(np.float32)
    g = rng.standard_normal(cloud.n).astype(np.float32)
    mu_d = torch.from_numpy(mu).to(dev)
    g_d = torch.from_numpy(g).to(dev)
    ref = torch.empty_like(mu_d)
    w.wnnc_winding_grad_x(ctx.handle, mu_d, None, 0.002, g_d, ref)
    got = torch.full_like(mu_d, float("nan"))
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    w.wnnc_winding_grad_x_noalloc(ctx.handle, mu_d, None, 0.002, g_d, got)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0, "device memory was allocated during the no-allocation call"
    a, b = got.cpu().numpy(), ref.cpu().numpy()
    assert np.array_equal(a, b), float(np.nanmax(np.abs(a - b)))
    if with_oracle:
        T = oracle_mod.Tree(x_or)
        m64, g64 = mu.astype(np.float64), g.astype(np.float64)
        G, magG, _, mgG = T.apply("G", m64, 0.002, 2.0, with_stats=True, with_margins=True)
        P, magP, _, mgP = T.apply("P", g64, 0.002, 2.0, with_stats=True, tvec=m64,
                                  with_margins=True)
        r = parity_bar.check("noalloc winding_grad_x", a, -g64[:, None] * G + P,
                             np.abs(g64) * magG + magP, np.hstack([mgG, mgP]))
        print(f"  {parity_bar.fmt(r)}", flush=True)
    ctx.close()


def test_noalloc_equals_the_allocating_entry_point(dev, oracle_mod):
    print("[case] noalloc knot20k then sphere2k", flush=True)
    _case(dev, synth.torus_knot(20000, 5, with_init=False), 1, oracle_mod, True)
    _case(dev, synth.fibonacci_sphere(2000, 0), 2, oracle_mod, True)


def test_noalloc_refuses_beyond_its_limit(dev):
    import torch
    import paper_2405_16634_amd as w
    n = w.NOALLOC_MAX_POINTS + 1
    print(f"[case] noalloc limit n={n}", flush=True)
    rng = np.random.default_rng(3)
    x = torch.from_numpy(rng.uniform(-0.9, 0.9, (n, 3)).astype(np.float32)).to(dev)
    ctx = w.Context(0)
    ctx.build(x)
    mu = torch.zeros(n, 3, device=dev)
    g = torch.zeros(n, device=dev)
    out = torch.zeros(n, 3, device=dev)
    with pytest.raises(w.WnncError) as e:
        w.wnnc_winding_grad_x_noalloc(ctx.handle, mu, None, 0.002, g, out)
    assert e.value.status == w.WNNC_EINVAL and "limit" in str(e.value)
    ctx.close()
