"""The opt-in check of the float inputs (WNNC_FLAG_CHECK_FINITE): a NaN or an
infinity in any checked input returns WNNC_ENUMERIC before any work, the
tree and results of earlier calls stay valid, finite inputs give the same
bits as without the check, and without the flag nothing is checked."""
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


def test_non_finite_inputs_are_reported(dev):
    import torch
    import paper_2405_16634_amd as w
    cloud = synth.fibonacci_sphere(2000, 0)
    print("[case] finite checks sphere2k", flush=True)
    ctx = w.Context(0)
    P = torch.from_numpy(cloud.points).to(dev)
    x, _ = ctx.normalize(P)
    ctx.build(x)
    mu = torch.from_numpy((cloud.normals * 1e-3).astype(np.float32)).to(dev)
    s_plain = ctx.winding(mu, 0.002).clone()
    ctx.set_flags(w.FLAG_CHECK_FINITE)
    assert torch.equal(ctx.winding(mu, 0.002), s_plain)

    def status(fn):
        with pytest.raises(w.WnncError) as e:
            fn()
        return e.value.status

    bad = mu.clone()
    bad[17, 1] = float("nan")
    assert status(lambda: ctx.winding(bad, 0.002)) == w.WNNC_ENUMERIC
    assert status(lambda: ctx.gradient(bad, 0.002)) == w.WNNC_ENUMERIC
    sig = torch.ones(cloud.n, device=dev)
    sig[5] = float("inf")
    assert status(lambda: ctx.winding(mu, 0.002, sigma=sig)) == w.WNNC_ENUMERIC
    s = torch.zeros(cloud.n, device=dev)
    s[-1] = float("-inf")
    assert status(lambda: ctx.adjoint(s, 0.002)) == w.WNNC_ENUMERIC
    assert status(lambda: ctx.orient(4, mu0=bad)) == w.WNNC_ENUMERIC
    Q = torch.zeros(10, 3, device=dev)
    Q[3, 0] = float("nan")
    assert status(lambda: ctx.winding_at(mu, 0.002, Q)) == w.WNNC_ENUMERIC
    assert status(lambda: ctx.winding_grad_x(mu, 0.002, s)) == w.WNNC_ENUMERIC
    Pb = x.clone()
    Pb[100, 2] = float("nan")
    assert status(lambda: ctx.build(Pb)) == w.WNNC_ENUMERIC
    # the tree of the last successful build is still in place
    assert torch.equal(ctx.winding(mu, 0.002), s_plain)
    # without the flag the inputs are not looked at
    ctx.set_flags(0)
    ctx.winding(bad, 0.002)
    torch.cuda.synchronize()
    ctx.close()
