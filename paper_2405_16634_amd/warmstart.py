"""Learned warm start: training-set generation, training and weights I/O.

Host orchestration only; every computation runs in the library's kernels
through the C ABI (orientation labels, k-nearest-neighbour features, the MLP
forward and gradient, Adam).

* Training clouds: a seeded mix of ellipsoid unions (1..8 members) and
  torus-knot tubes ((p,q) in {(2,3),(2,5),(3,4),(3,5)}, tube radius
  U[0.03, 0.08], density ratio U[1, 10]) of U{n_lo..n_hi} points, each under a
  uniform random rotation.
* Labels: unit normals of the plain method (Alg. 3 from mu = 0, 40
  iterations, default widths), computed for many clouds at once on a batched
  forest.
* Training: full-batch Adam on mean(1 - cos(prediction, label)).

``python -m paper_2405_16634_amd.warmstart --out PATH`` trains and writes the
parameter vector (7491 FP32 values) as a .npy file.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

from . import MLP_PARAMS, Context, wnnc_mlp_adam, wnnc_mlp_grad

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "data", "warmstart_mlp.npy")


def _rotate(points, normals, rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    R = np.array([
        [a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
        [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
        [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])
    return (points @ R.T).astype(np.float32), (normals @ R.T).astype(np.float32)


def training_clouds(count: int, seed: int = 1000, n_lo: int = 10000, n_hi: int = 50000):
    """Seeded synthetic training clouds (points only; labels come from the
    plain method)."""
    import synth
    out = []
    for k in range(count):
        rng = np.random.default_rng(seed + k)
        n = int(rng.integers(n_lo, n_hi + 1))
        if k % 2 == 0:
            c = synth.ellipsoid_union(n, seed=seed + k, members=int(rng.integers(1, 9)),
                                      noise=0.0, with_init=False)
        else:
            p, q = [(2, 3), (2, 5), (3, 4), (3, 5)][int(rng.integers(0, 4))]
            c = synth.torus_knot(n, seed=seed + k, outlier_frac=0.0, p=p, q=q,
                                 tube=float(rng.uniform(0.03, 0.08)),
                                 density_ratio=float(rng.uniform(1.0, 10.0)), with_init=False,
                                 samples=8000)
        pts, _ = _rotate(c.points.astype(np.float64), c.normals.astype(np.float64), rng)
        out.append(pts)
    return out


def label_and_features(clouds, device: int = 0, group_points: int = 3_000_000, iters: int = 40,
                       w1: float = 0.002, w2: float = 0.016):
    """Features (N,48) and plain-method unit normals (N,3) of all clouds, as
    CUDA tensors; clouds are processed as batched forests of about
    group_points points."""
    feats, labels = [], []
    i = 0
    while i < len(clouds):
        j = i
        tot = 0
        while j < len(clouds) and (tot == 0 or tot + len(clouds[j]) <= group_points):
            tot += len(clouds[j])
            j += 1
        grp = clouds[i:j]
        off = np.concatenate([[0], np.cumsum([len(c) for c in grp])]).astype(np.int64)
        ctx = Context(device)
        P = torch.from_numpy(np.concatenate(grp)).to(f"cuda:{device}")
        x, _ = ctx.normalize_batched(P, off)
        ctx.build_batched(x, off)
        mu = ctx.orient(iters, w1, w2)
        labels.append(ctx.normals(mu))
        feats.append(ctx.features())
        torch.cuda.synchronize()
        ctx.close()
        i = j
    return torch.cat(feats), torch.cat(labels)


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases (layout of include/wnnc.h)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((48, 64), (64, 64), (64, 3)):
        parts.append(rng.standard_normal((fan_in, fan_out)).reshape(-1) * np.sqrt(2.0 / fan_in))
        parts.append(np.zeros(fan_out))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == MLP_PARAMS
    return p


def train(feat, labels, steps: int = 800, lr: float = 3e-3, seed: int = 0, device: int = 0,
          log_every: int = 100, params=None):
    """Full-batch Adam with a cosine learning-rate decay.  Returns (params as
    a CUDA tensor, loss history)."""
    ctx = Context(device)
    dev = f"cuda:{device}"
    p = torch.from_numpy(init_params(seed) if params is None else np.asarray(params, np.float32)).to(dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    g = torch.empty_like(p)
    hist = []
    for step in range(1, steps + 1):
        want = step == 1 or step % log_every == 0 or step == steps
        loss = wnnc_mlp_grad(ctx.handle, p, feat, labels, g, with_loss=want)
        if want:
            hist.append((step, loss))
        lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * (step - 1) / steps))
        wnnc_mlp_adam(ctx.handle, p, m, v, g, step, max(lr_t, 1e-5))
    final = wnnc_mlp_grad(ctx.handle, p, feat, labels, g, with_loss=True)
    hist.append((steps + 1, final))
    ctx.close()
    return p, hist


def save_params(p, path: str = DEFAULT_WEIGHTS, meta: dict | None = None) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    arr = p.detach().cpu().numpy().astype(np.float32) if isinstance(p, torch.Tensor) else np.asarray(p, np.float32)
    np.save(path, arr)
    if meta is not None:
        with open(os.path.splitext(path)[0] + ".json", "w") as f:
            json.dump(meta, f, indent=1)


def load_params(path: str = DEFAULT_WEIGHTS, device: int = 0):
    arr = np.load(path, allow_pickle=False).astype(np.float32)
    if arr.size != MLP_PARAMS:
        raise ValueError(f"{path}: expected {MLP_PARAMS} parameters, got {arr.size}")
    return torch.from_numpy(arr).to(f"cuda:{device}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--clouds", type=int, default=96)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--steps", type=int, default=800)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args()
    t0 = time.time()
    clouds = training_clouds(args.clouds, args.seed)
    t1 = time.time()
    print(f"generated {len(clouds)} clouds, {sum(len(c) for c in clouds)} points in {t1 - t0:.1f} s",
          flush=True)
    feat, lab = label_and_features(clouds)
    t2 = time.time()
    print(f"labels and features in {t2 - t1:.1f} s", flush=True)
    p, hist = train(feat, lab, args.steps, args.lr)
    t3 = time.time()
    for s, l in hist:
        print(f"  step {s}: loss {l:.5f}", flush=True)
    print(f"trained in {t3 - t2:.1f} s", flush=True)
    save_params(p, args.out, dict(clouds=args.clouds, seed=args.seed, steps=args.steps, lr=args.lr,
                                  points=int(feat.shape[0]), final_loss=hist[-1][1]))


if __name__ == "__main__":
    main()
