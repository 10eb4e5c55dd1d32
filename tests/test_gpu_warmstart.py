"""Warm-start kernels against the FP64 reference (oracle/mlp.py):
k-nearest neighbours on the octree, neighbourhood features, the BF16 MFMA
network forward and gradient, and the Adam step."""
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


def _t(a, dev, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype or np.float32)).to(dev)


def test_knn_and_features(dev):
    import torch
    import paper_2405_16634_amd as w
    from oracle import mlp
    rng = np.random.default_rng(3)
    clouds = [synth.torus_knot(8000, 5, with_init=False).points,
              rng.uniform(-1, 1, (5, 3)).astype(np.float32),
              synth.fibonacci_sphere(1500, 0).points]
    off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])]).astype(np.int64)
    ctx = w.Context(0)
    x, _ = ctx.normalize_batched(_t(np.concatenate(clouds), dev), off)
    ctx.build_batched(x, off)
    n = int(off[-1])
    feat = torch.empty(n, 48, device=dev)
    nbr = torch.empty(n, 16, device=dev, dtype=torch.int32)
    w.wnnc_knn_features(ctx.handle, feat, nbr)
    xh = x.cpu().numpy().astype(np.float64)
    gi = nbr.cpu().numpy().astype(np.int64)
    groups = np.repeat(np.arange(len(clouds)), np.diff(off))
    oi, od2 = mlp.knn(xh, 16, groups)
    # distances are unique even where equal distances order differently
    gd2 = np.where(gi >= 0, ((xh[np.maximum(gi, 0)] - xh[:, None, :]) ** 2).sum(2), np.inf)
    fin = np.isfinite(od2)
    assert np.array_equal(np.isfinite(gd2), fin)
    assert np.allclose(np.sort(gd2, 1)[fin], od2[fin], rtol=1e-5, atol=1e-12)
    same = (gi == oi).all(1).mean()
    print(f"  knn index agreement {same:.5f}", flush=True)
    assert same > 0.99
    # features of the device's neighbour lists
    ref = mlp.features(xh, gi)
    assert np.max(np.abs(feat.cpu().numpy() - ref)) < 2e-5
    ctx.close()


def test_mlp_forward_grad_adam(dev):
    import torch
    import paper_2405_16634_amd as w
    from oracle import mlp
    rng = np.random.default_rng(9)
    n = 5000
    X = rng.standard_normal((n, 48)).astype(np.float32)
    L = rng.standard_normal((n, 3))
    L = (L / np.linalg.norm(L, axis=1, keepdims=True)).astype(np.float32)
    p = mlp.init_params(7).astype(np.float32)
    ctx = w.Context(0)
    P, Xd, Ld = _t(p, dev), _t(X, dev), _t(L, dev)
    out = torch.empty(n, 3, device=dev)
    w.wnnc_mlp_forward(ctx.handle, P, Xd, out)
    _, _, y = mlp.forward(p.astype(np.float64), X, rounding=True)
    yn = y / np.linalg.norm(y, axis=1, keepdims=True)
    cosang = (out.cpu().numpy() * yn).sum(1)
    print(f"  forward min cos {cosang.min():.8f}", flush=True)
    assert cosang.min() > 1 - 1e-5
    grad = torch.empty(w.MLP_PARAMS, device=dev)
    loss = w.wnnc_mlp_grad(ctx.handle, P, Xd, Ld, grad)
    rl, rg = mlp.loss_grad(p.astype(np.float64), X, L.astype(np.float64), rounding=True)
    g = grad.cpu().numpy()
    assert abs(loss - rl) < 1e-5
    o = 0
    for name, shape in mlp.SIZES:
        k = int(np.prod(shape))
        err = np.linalg.norm(g[o:o + k] - rg[o:o + k]) / np.linalg.norm(rg[o:o + k])
        print(f"  grad {name}: rel_l2={err:.2e}", flush=True)
        assert err < 1e-3, name
        o += k
    m = torch.zeros_like(grad)
    v = torch.zeros_like(grad)
    w.wnnc_mlp_adam(ctx.handle, P, m, v, grad, 1, 1e-3)
    p1, _, _ = mlp.adam(p.astype(np.float64), np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS),
                        g.astype(np.float64), 1, 1e-3)
    assert np.max(np.abs(P.cpu().numpy() - p1)) < 1e-6
    ctx.close()


def test_training_reduces_the_loss(dev):
    import torch
    import paper_2405_16634_amd as w
    from oracle import mlp
    rng = np.random.default_rng(2)
    n = 20000
    X = rng.standard_normal((n, 48)).astype(np.float32)
    # a learnable target: a fixed linear map of the features, normalized
    A = rng.standard_normal((48, 3))
    L = X @ A
    L = (L / np.linalg.norm(L, axis=1, keepdims=True)).astype(np.float32)
    p = _t(mlp.init_params(1), dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    g = torch.empty_like(p)
    ctx = w.Context(0)
    Xd, Ld = _t(X, dev), _t(L, dev)
    first = w.wnnc_mlp_grad(ctx.handle, p, Xd, Ld, g)
    for step in range(1, 201):
        w.wnnc_mlp_grad(ctx.handle, p, Xd, Ld, g, with_loss=False)
        w.wnnc_mlp_adam(ctx.handle, p, m, v, g, step, 3e-3)
    last = w.wnnc_mlp_grad(ctx.handle, p, Xd, Ld, g)
    print(f"  loss {first:.4f} -> {last:.4f}", flush=True)
    assert last < 0.25 * first
    ctx.close()
