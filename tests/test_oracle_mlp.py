"""Pins of the warm-start reference (oracle/mlp.py) against what the
mathematics fixes: finite differences of the FP64 network, the BF16
rounding rule on representable values, neighbour counts on a lattice, and
the known first Adam step."""
import numpy as np
import pytest

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


def _hand_network():
    """A network whose every value is worked out by hand (all of them exact
    in BF16): one input row x with x0 = 2, x1 = 1/4, x5 = 3/2, x7 = 3/4.
      layer 1 (W1[in][out], b1 = -1/2): h1_0 = relu(2 - 1/2) = 3/2,
        h1_1 = relu(1/4 - 1/2) = 0 (the ReLU cuts), h1_7 = relu(x5 - 1/2) = 1
        (W1[5][7]: input 5 feeds hidden unit 7), the rest relu(-1/2) = 0;
      layer 2: h2_0 = 2 h1_0 = 3, h2_1 = h1_1 + 1/4 = 1/4, h2_3 = h1_7 + 1/2
        = 3/2, h2_4 = relu(-4 h1_0 + 1) = relu(-5) = 0;
      layer 3: y = (h2_0, 2 h2_3 + h2_4 + 1, 4 h2_1 - 1) = (3, 4, 0)."""
    d = {name: np.zeros(shape) for name, shape in mlp.SIZES}
    d["W1"][0, 0] = 1.0
    d["W1"][1, 1] = 1.0
    d["W1"][5, 7] = 1.0
    d["b1"][:] = -0.5
    d["W2"][0, 0] = 2.0
    d["W2"][1, 1] = 1.0
    d["W2"][7, 3] = 1.0
    d["W2"][0, 4] = -4.0
    d["b2"][1], d["b2"][3], d["b2"][4] = 0.25, 0.5, 1.0
    d["W3"][0, 0] = 1.0
    d["W3"][3, 1] = 2.0
    d["W3"][4, 1] = 1.0
    d["W3"][1, 2] = 4.0
    d["b3"][:] = [0.0, 1.0, -1.0]
    X = np.zeros((1, 48))
    X[0, 0], X[0, 1], X[0, 5], X[0, 7] = 2.0, 0.25, 1.5, 0.75
    return mlp.pack(d), X


def test_forward_by_hand():
    """The hand network gives y = (3, 4, 0) exactly, with and without the
    BF16 rounding (every operand is a BF16 value).  A missing ReLU (either
    layer), a transposed weight matrix or a dropped bias changes y."""
    p, X = _hand_network()
    for rounding in (False, True):
        h1, h2, y = mlp.forward(p, X, rounding=rounding)
        assert np.array_equal(y[0], [3.0, 4.0, 0.0])
        assert h1[0, 0] == 1.5 and h1[0, 1] == 0.0 and h1[0, 7] == 1.0
        assert np.count_nonzero(h1) == 2
        assert h2[0, 0] == 3.0 and h2[0, 1] == 0.25 and h2[0, 3] == 1.5 and h2[0, 4] == 0.0


def test_loss_and_gradient_by_hand():
    """With label (1, 0, 0): cos(y, L) = 3/5, loss 2/5.  d(1 - cos)/dy =
    -(L/|y| - y (y.L)/|y|^3) = (-0.128, 0.096, 0) = grad b3; back through the
    layers by hand: grad W3[0][0] = h2_0 dy_0 = -0.384; d2_3 = 2 dy_1 = 0.192
    (W3[3][1] = 2), so grad b2_3 = 0.192 and grad W2[7][3] = h1_7 d2_3 =
    0.192; d2_4 = 0 (the ReLU cut h2_4), so grad b2_4 = 0; d1_7 = d2_3 = 0.192,
    so grad W1[5][7] = x5 d1_7 = 0.288; d1_0 = 2 d2_0 = -0.256, so
    grad W1[0][0] = x0 d1_0 = -0.512; d1_1 = 0 (ReLU), so grad b1_1 = 0."""
    p, X = _hand_network()
    L = np.array([[1.0, 0.0, 0.0]])
    loss, g = mlp.loss_grad(p, X, L, rounding=False)
    assert loss == pytest.approx(0.4, abs=1e-15)
    gd = mlp.unpack(g)
    assert np.allclose(gd["b3"], [-0.128, 0.096, 0.0], rtol=0, atol=1e-15)
    assert gd["W3"][0, 0] == pytest.approx(-0.384, abs=1e-15)
    assert gd["b2"][3] == pytest.approx(0.192, abs=1e-15)
    assert gd["W2"][7, 3] == pytest.approx(0.192, abs=1e-15)
    assert gd["b2"][4] == 0.0
    assert gd["W1"][5, 7] == pytest.approx(0.288, abs=1e-15)
    assert gd["W1"][0, 0] == pytest.approx(-0.512, abs=1e-15)
    assert gd["b1"][1] == 0.0 and gd["b1"][7] == pytest.approx(0.192, abs=1e-15)
