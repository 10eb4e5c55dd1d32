"""The adjoint kernel behind torch.autograd (Sec. 4.5: A^T is the backward
of A), checked against central finite differences and the FP64 oracle.

Workload: a 5,000-point subset of the torus-knot cloud (the first 5,000 of a
seeded permutation of its surface points), as a cloud of its own.
"""
import numpy as np
import pytest

import parity_bar
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_2405_16634_amd as w
    knot = synth.torus_knot(500000, 3)
    surf = np.where(np.isfinite(knot.normals).all(axis=1))[0]
    sub = np.random.default_rng(17).permutation(surf)[:5000]
    pts = knot.points[sub]
    nrm = knot.normals[sub]
    dev = torch.device("cuda:0")
    x_or, _, sc = oracle.normalize(pts)
    ctx = w.Context(0)
    x_dev, _ = ctx.normalize(torch.from_numpy(pts).to(dev))
    ctx.build(x_dev)
    area = knot.area * len(sub) / knot.n
    mu = (nrm * (area * sc * sc / len(sub))).astype(np.float32)
    yield dict(ctx=ctx, x=x_or.astype(np.float64), mu=mu, dev=dev, n=len(sub))
    ctx.close()


def _t(a, dev, grad=False):
    import torch
    return torch.tensor(np.asarray(a, np.float32), device=dev, requires_grad=grad)


def test_winding_backward_is_the_oracle_adjoint(setup, oracle_mod):
    from paper_2405_16634_amd import autograd as ag
    ctx, x, mu, dev = setup["ctx"], setup["x"], setup["mu"], setup["dev"]
    rng = np.random.default_rng(0)
    g = rng.standard_normal(setup["n"]).astype(np.float32)
    m = _t(mu, dev, grad=True)
    s = ag.winding(ctx, m, 0.002)
    (s * _t(g, dev)).sum().backward()
    got = m.grad.cpu().numpy().astype(np.float64)
    T = oracle_mod.Tree(x)
    ref, mag, _, mg = T.apply("AT", g.astype(np.float64), 0.002, 2.0, with_stats=True,
                              with_margins=True)
    r = parity_bar.check("A backward", got, ref, mag, mg)
    print(f"  A backward: {parity_bar.fmt(r)}", flush=True)


def test_adjoint_and_gradient_backward(setup, oracle_mod):
    from paper_2405_16634_amd import autograd as ag
    ctx, x, mu, dev = setup["ctx"], setup["x"], setup["mu"], setup["dev"]
    rng = np.random.default_rng(1)
    s0 = rng.standard_normal(setup["n"]).astype(np.float32)
    v = (rng.standard_normal((setup["n"], 3)) * 1e-4).astype(np.float32)
    T = oracle_mod.Tree(x)
    # d<v, A^T s>/ds = A v
    st = _t(s0, dev, grad=True)
    (ag.adjoint(ctx, st, 0.002) * _t(v, dev)).sum().backward()
    ref, mag, _, mg = T.apply("A", v.astype(np.float64), 0.002, 2.0, with_stats=True,
                              with_margins=True)
    r = parity_bar.check("A^T backward", st.grad.cpu().numpy(), ref, mag, mg)
    print(f"  A^T backward: {parity_bar.fmt(r)}", flush=True)
    # d<v, grad F(mu)>/dmu = -G v
    m = _t(mu, dev, grad=True)
    (ag.gradient(ctx, m, 0.002) * _t(v, dev)).sum().backward()
    ref, mag, _, mg = T.apply("G", v.astype(np.float64), 0.002, 2.0, with_stats=True,
                              with_margins=True)
    r = parity_bar.check("grad F backward", m.grad.cpu().numpy(), -ref, mag, mg)
    print(f"  grad F backward: {parity_bar.fmt(r)}", flush=True)


def test_energy_gradient_is_minus_two_r(setup, oracle_mod):
    """E = ||A mu - b||^2 (b = 1/2) and dE/dmu = -2 r with r from Alg. 2, both
    evaluated by the library (wnnc_energy) and reached through autograd."""
    from paper_2405_16634_amd import autograd as ag
    ctx, x, mu, dev = setup["ctx"], setup["x"], setup["mu"], setup["dev"]
    m = _t(mu, dev, grad=True)
    E = ag.pgr_energy(ctx, m, 0.002)
    (3.0 * E).backward()  # a chain-rule factor other than 1
    T = oracle_mod.Tree(x)
    s, smag, _, smg = T.apply("A", mu.astype(np.float64), 0.002, 2.0, with_stats=True,
                              with_margins=True)
    s_gpu = ag.winding(ctx, _t(mu, dev), 0.002).detach().cpu().numpy().astype(np.float64)
    parity_bar.check("energy forward A", s_gpu, s, smag, smg)
    # E is the FP64 sum of the device's FP32 rho_i^2 (rho rounded from the
    # FP64 sum, s_gpu from the same sum: within an ulp of each other)
    rho = 0.5 - s_gpu
    assert float(E) == pytest.approx(float((rho * rho).sum()), rel=1e-6)
    assert float(E) == pytest.approx(float(((0.5 - s) ** 2).sum()), rel=1e-4)
    # the backward applies A^T to -6 rho; compare with the oracle's A^T of
    # the same vector so only the adjoint is under test
    ref, mag, _, mg = T.apply("AT", -6.0 * rho, 0.002, 2.0, with_stats=True, with_margins=True)
    r = parity_bar.check("energy backward", m.grad.cpu().numpy(), ref, mag, mg)
    print(f"  energy backward: {parity_bar.fmt(r)}", flush=True)
    # and against the oracle's own residual: 3 dE/dmu = -6 r = 6 A^T (A mu - b)
    ref2 = T.apply("AT", 6.0 * (s - 0.5), 0.002)
    l2 = np.linalg.norm(m.grad.cpu().numpy() - ref2) / np.linalg.norm(ref2)
    assert l2 < 1e-3


def test_central_finite_differences(setup, oracle_mod):
    """Central differences with h = 1e-3 relative to the RMS |mu|.

    Exact limit (c huge, the treecode is the direct sum and A is linear):
    the autograd gradient matches finite differences of the FP64 direct sum
    and of the device forward itself.  Paper setting (c = 2): it matches
    finite differences of the FP64 direct sum within the treecode's error."""
    import torch
    import paper_2405_16634_amd as w
    from paper_2405_16634_amd import autograd as ag
    x, mu, dev, n = setup["x"], setup["mu"], setup["dev"], setup["n"]
    rng = np.random.default_rng(2)
    g = rng.standard_normal(n)
    v = rng.standard_normal((n, 3))
    h = 1e-3 * float(np.sqrt((mu.astype(np.float64) ** 2).sum(1).mean()))
    fd_exact = (g @ oracle_mod.direct("A", x, mu + h * v, 0.002)
                - g @ oracle_mod.direct("A", x, mu - h * v, 0.002)) / (2 * h)
    # the oracle treecode's own deviation from the exact derivative at c = 2
    T = oracle_mod.Tree(x)
    dd_tree = float((T.apply("AT", g, 0.002, 2.0) * v).sum())
    for c in (1e6, 2.0):
        ctx = w.Context(0)
        ctx.build(_t(x, dev), c)
        m = _t(mu, dev, grad=True)
        (ag.winding(ctx, m, 0.002) * _t(g, dev)).sum().backward()
        dd = float((m.grad.cpu().numpy().astype(np.float64) * v).sum())
        print(f"  c={c}: autograd={dd:.6e} fd_exact={fd_exact:.6e} oracle_tree={dd_tree:.6e}", flush=True)
        if c > 1e5:
            # FP32 sums of ~5000 random-sign terms per target
            assert abs(dd - fd_exact) <= 1e-3 * abs(fd_exact)
            with torch.no_grad():
                lp = float((ag.winding(ctx, _t(mu + h * v, dev), 0.002).double().cpu().numpy() * g).sum())
                lm = float((ag.winding(ctx, _t(mu - h * v, dev), 0.002).double().cpu().numpy() * g).sum())
            fd_dev = (lp - lm) / (2 * h)
            assert abs(dd - fd_dev) <= 2e-2 * abs(fd_exact)
        else:
            # same deviation from the exact derivative as the FP64 treecode
            assert abs(dd - dd_tree) <= 1e-3 * abs(fd_exact)
        ctx.close()
