"""Pins of the warm-start reference (oracle/mlp.py) against what the
mathematics fixes: finite differences of the FP64 network, the BF16
rounding rule on representable values, neighbour counts on a lattice, and
the known first Adam step."""
import numpy as np

from oracle import mlp


def test_parameter_count():
    assert mlp.N_PARAMS == 7491


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(3)
    X = rng.standard_normal((40, 48))
    L = rng.standard_normal((40, 3))
    L /= np.linalg.norm(L, axis=1, keepdims=True)
    _, g = mlp.loss_grad(p, X, L, rounding=False)
    h = 1e-6
    for k in rng.choice(mlp.N_PARAMS, 60, replace=False):
        e = np.zeros_like(p)
        e[k] = h
        fd = (mlp.loss_grad(p + e, X, L, rounding=False)[0]
              - mlp.loss_grad(p - e, X, L, rounding=False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])), k


def test_bf16_rounding_rule():
    # values exactly representable in BF16 are unchanged; halfway cases go
    # to the even neighbour; the rest to the nearest
    exact = np.array([1.0, -2.5, 0.0078125, 3.0e38 // 1e30 * 1e30])
    assert np.all(mlp.bf16(exact[:3]) == exact[:3])
    one_ulp = 2.0 ** -7  # BF16 spacing just above 1
    assert mlp.bf16(1.0 + one_ulp / 2) == 1.0            # tie -> even (1.0)
    assert mlp.bf16(1.0 + 1.5 * one_ulp) == 1.0 + 2 * one_ulp  # tie -> even
    assert mlp.bf16(1.0 + 0.6 * one_ulp) == 1.0 + one_ulp


def test_knn_on_a_lattice():
    """On a cubic lattice of spacing h an interior point has 6 neighbours at
    distance h and 12 at h sqrt 2."""
    h = 0.1
    g = np.arange(5) * h
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    idx, d2 = mlp.knn(x, 16)
    centre = np.where((x == 2 * h).all(1))[0][0]
    d = np.sqrt(d2[centre])
    assert np.allclose(d[:6], h) and np.allclose(d[6:16], h * np.sqrt(2))
    f = mlp.features(x, idx)
    assert f.shape == (len(x), 48)
    rms = np.sqrt((f[centre].reshape(16, 3) ** 2).sum(1).mean())
    assert abs(rms - 1.0) < 1e-12


def test_knn_groups_and_small_clouds():
    x = np.array([[0, 0, 0], [1, 0, 0], [5, 5, 5]], dtype=np.float64)
    idx, _ = mlp.knn(x, 16, groups=np.array([0, 0, 1]))
    assert idx[0, 0] == 1 and idx[1, 0] == 0 and np.all(idx[0, 1:] == -1)
    assert np.all(idx[2] == -1)
    f = mlp.features(x, idx)
    assert np.all(f[2] == 0)


def test_first_adam_step_is_lr_times_sign():
    """With bias correction the first step moves every parameter by lr in
    the direction opposite to its gradient (up to eps)."""
    rng = np.random.default_rng(1)
    p = rng.standard_normal(10)
    g = rng.standard_normal(10)
    p1, m, v = mlp.adam(p, np.zeros(10), np.zeros(10), g, 1, lr=0.01, eps=1e-12)
    assert np.allclose(p1 - p, -0.01 * np.sign(g), atol=1e-9)
