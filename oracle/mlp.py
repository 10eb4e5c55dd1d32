"""FP64 reference of the warm-start network and its features (test
infrastructure only).

* ``knn``: the k nearest other points of each point, by brute force
  (ties by index).
* ``features``: offsets to the 16 nearest neighbours, nearest first, divided
  by their RMS length (48 values per point).
* ``forward`` / ``loss_grad``: the 48 -> 64 -> 64 -> 3 ReLU network and the
  gradient of mean(1 - cos(y, label)).  With ``rounding=True`` every matrix
  product takes its operands rounded to BF16 (round to nearest even), as the
  device does; the products, biases, loss and the chain rule are FP64.  With
  ``rounding=False`` it is the plain FP64 network, whose gradient is pinned
  against finite differences.
* ``adam``: one bias-corrected Adam step (Kingma & Ba 2015).

Parameter vector layout: W1 [48][64], b1 [64], W2 [64][64], b2 [64],
W3 [64][3], b3 [3], row-major [in][out].
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 48, 64, 3
SIZES = [("W1", (N_IN, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("W3", (N_HID, N_OUT)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def bf16(x):
    """Round to FP32, then to BF16 with round-to-nearest-even; as float64."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed: int = 0):
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SIZES:
        if name.startswith("W"):
            d[name] = rng.standard_normal(shape) * np.sqrt(2.0 / shape[0])
        else:
            d[name] = np.zeros(shape)
    return pack(d)


def knn(x, k: int = 16, groups=None):
    """Indices (n, k) of the k nearest other points (ties by index), -1 where
    a group has fewer than k + 1 points.  groups: per-point group labels
    (neighbours only within a group)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    idx = np.full((n, k), -1, np.int64)
    d2 = np.full((n, k), np.inf)
    g = np.zeros(n, np.int64) if groups is None else np.asarray(groups)
    for lab in np.unique(g):
        sel = np.where(g == lab)[0]
        xs = x[sel]
        for a in range(0, len(sel), 512):
            blk = xs[a:a + 512]
            dd = ((blk[:, None, :] - xs[None, :, :]) ** 2).sum(2)
            dd[np.arange(len(blk)), a + np.arange(len(blk))] = np.inf
            order = np.lexsort((np.broadcast_to(sel, dd.shape), dd), axis=1)[:, :k]
            m = min(k, len(sel) - 1)
            idx[sel[a:a + 512], :m] = sel[order[:, :m]]
            d2[sel[a:a + 512], :m] = np.take_along_axis(dd, order[:, :m], axis=1)
    return idx, d2


def features(x, idx):
    """Offsets to the neighbours idx (n,16), divided by their RMS length."""
    x = np.asarray(x, dtype=np.float64)
    valid = idx >= 0
    off = np.where(valid[:, :, None], x[np.maximum(idx, 0)] - x[:, None, :], 0.0)
    cnt = valid.sum(1)
    rms = np.sqrt((off ** 2).sum((1, 2)) / np.maximum(cnt, 1))
    inv = np.where(rms > 0, 1.0 / np.where(rms > 0, rms, 1.0), 0.0)
    return (off * inv[:, None, None]).reshape(len(x), -1)


def forward(p, X, rounding: bool = True):
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    w = unpack(p)
    h1 = np.maximum(r(X) @ r(w["W1"]) + w["b1"], 0.0)
    h2 = np.maximum(r(h1) @ r(w["W2"]) + w["b2"], 0.0)
    y = r(h2) @ r(w["W3"]) + w["b3"]
    return h1, h2, y


def loss_grad(p, X, L, rounding: bool = True):
    """(loss, gradient) of mean_i (1 - cos(y_i, L_i))."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    w = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    n = len(X)
    h1, h2, y = forward(p, X, rounding)
    yy = np.linalg.norm(y, axis=1)
    ll = np.linalg.norm(L, axis=1)
    ok = (yy > 0) & (ll > 0)
    yl = (y * L).sum(1)
    cos = np.where(ok, yl / np.where(ok, yy * ll, 1.0), 0.0)
    loss = float((1.0 - cos).mean())
    a = np.where(ok, 1.0 / np.where(ok, yy * ll, 1.0), 0.0)
    b = np.where(ok, yl / np.where(ok, yy ** 3 * ll, 1.0), 0.0)
    dy = -(L * a[:, None] - y * b[:, None]) / n
    g = {}
    g["W3"] = r(h2).T @ r(dy)
    g["b3"] = dy.sum(0)
    d2 = (r(dy) @ r(w["W3"]).T) * (h2 > 0)
    g["W2"] = r(h1).T @ r(d2)
    g["b2"] = d2.sum(0)
    d1 = (r(d2) @ r(w["W2"]).T) * (h1 > 0)
    g["W1"] = r(X).T @ r(d1)
    g["b1"] = d1.sum(0)
    return loss, pack(g)


def adam(p, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
