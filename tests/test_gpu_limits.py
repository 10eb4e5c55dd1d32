"""Size limits of the tree, at their boundaries on the device: a build whose
tree has more nodes than the 32-bit record offsets address is refused, and
so is the far field of order > 0 on a tree beyond the 32-bit offsets of its
moments, both with WNNC_EINVAL and a message (no wrapped offsets).  Uniform
random clouds in [-1, 1]^3 of tens of millions of points, seeded."""
import pytest

pytestmark = pytest.mark.gpu

MAX_NODES = 1 << 26
MAX_HI_NODES = (1 << 32) // 96


def _cloud(n, seed):
    import torch
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    return torch.rand((n, 3), device="cuda:0", generator=g) * 1.8 - 0.9


def test_far_field_node_limit():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_16634_amd as w
    n = 36_000_000
    print(f"[case] far-field node limit, uniform cloud of {n} points", flush=True)
    ctx = w.Context(0)
    ctx.build(_cloud(n, 5))
    m = ctx.stats()["n_nodes"]
    print(f"  nodes {m}", flush=True)
    assert MAX_HI_NODES < m <= MAX_NODES
    with pytest.raises(w.WnncError) as e:
        ctx.set_far_field(2, False)
    assert e.value.status == w.WNNC_EINVAL
    assert ctx.far_field() == (0, False)
    # the far field set first: the build of the large tree is refused
    small = _cloud(1000, 6)
    ctx.build(small)
    ctx.set_far_field(2, True)
    with pytest.raises(w.WnncError) as e:
        ctx.build(_cloud(n, 5))
    assert e.value.status == w.WNNC_EINVAL
    # the context stays usable
    ctx.build(small)
    mu = torch.zeros((1000, 3), device="cuda:0")
    mu[:, 2] = 1e-3
    assert bool(torch.isfinite(ctx.winding(mu, 0.002)).all())
    ctx.close()
    torch.cuda.empty_cache()


def test_node_limit():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_16634_amd as w
    n = 64_000_000
    print(f"[case] node limit, uniform cloud of {n} points", flush=True)
    ctx = w.Context(0)
    with pytest.raises(w.WnncError) as e:
        ctx.build(_cloud(n, 7))
    assert e.value.status == w.WNNC_EINVAL
    assert "nodes" in str(e.value)
    ctx.close()
    torch.cuda.empty_cache()
