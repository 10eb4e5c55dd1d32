"""Alg. 2 (grad_step) and Alg. 3 (WNNC iteration with smoothing) in FP64.

Test infrastructure only.  The operators come from either the exact direct
sums or the paper's treecode, both in this package.

Alg. 3, per iteration i = 1..n:
  w = w2 (n-i)/(n-1) + w1 (i-1)/(n-1)              (width schedule)
  mu <- grad_step(mu; A_w, b),  b = (1/2, ..., 1/2)  (Alg. 2)
  mu^ <- G_w(mu)                                     (WNNC update)
  mu_i <- mu^_i |mu_i| / |mu^_i|                     (rescale)
starting from mu = 0 (Sec. 4.3).

Alg. 2 for E(mu) = ||A mu - b||^2:
  r <- A^T b - A^T A mu,  alpha <- r^T r / (r^T A^T A r),  mu <- mu + alpha r

Readings (where the paper leaves a choice):
* r is evaluated as one adjoint application to the residual, r = A^T(b - A mu),
  and r^T A^T A r as |A r|^2, so one step costs A, A^T, A.  With the exact
  operators this is the printed formula; with the treecode it is the natural
  way to apply it (the treecode adjoint is not linear in its argument).
* alpha = 0 when |A r|^2 = 0.
* rescale keeps mu_i unchanged when |mu^_i| is 0 or not finite, and a zero
  mu_i stays zero.
* n = 1 uses w = w1.

Variants (other width schedules, Sec. 5.5.1; fixed areas, Sec. 6.1.1):
* the paper reports cosine and exponential schedules behaving like the
  linear one, without formulas; read as the smooth decreasing curves from w2
  (i = 1) to w1 (i = n):
    cosine      w = w1 + (w2 - w1) (1 + cos(pi t)) / 2
    exponential w = w2 (w1 / w2)^t          (w1, w2 > 0)
  with t = (i - 1) / (n - 1);
* with given areas sigma, the rescale sets |mu_i| = sigma_i:
  mu_i <- mu^_i sigma_i / |mu^_i| (kept when |mu^_i| is 0 or not finite).
"""
from __future__ import annotations

import numpy as np


def width_schedule(i: int, n: int, w1: float, w2: float, mode: str = "linear") -> float:
    """Width of iteration i (1-based) of n: the linear schedule of Alg. 3, or
    the cosine / exponential variants (module docstring)."""
    if n <= 1:
        return float(w1)
    t = (i - 1) / (n - 1)
    if mode == "linear":
        return w2 * (n - i) / (n - 1) + w1 * (i - 1) / (n - 1)
    if mode == "cosine":
        return w1 + (w2 - w1) * (1.0 + np.cos(np.pi * t)) / 2.0
    if mode == "exponential":
        if not (w1 > 0 and w2 > 0):
            raise ValueError("the exponential schedule needs w1, w2 > 0")
        return w2 * (w1 / w2) ** t
    raise ValueError(mode)


def rescale(mu, mu_hat, areas=None):
    """mu_i <- mu^_i |mu_i| / |mu^_i| (Alg. 3), or mu^_i sigma_i / |mu^_i|
    with given areas (Sec. 6.1.1); kept when |mu^_i| is 0 or not finite."""
    mu = np.asarray(mu, dtype=np.float64)
    mu_hat = np.asarray(mu_hat, dtype=np.float64)
    nh = np.linalg.norm(mu_hat, axis=1)
    nm = np.linalg.norm(mu, axis=1) if areas is None else np.asarray(areas, dtype=np.float64)
    ok = np.isfinite(nh) & (nh > 0)
    out = mu.copy()
    out[ok] = mu_hat[ok] * (nm[ok] / nh[ok])[:, None]
    return out


class _Ops:
    """A, A^T, G at width w through the chosen backend."""

    def __init__(self, x, backend, c=2.0, max_depth=15, leaf_cap=1, order=0, wsafe=False):
        from . import Tree, direct
        self.x = np.asarray(x, dtype=np.float64)
        self.backend = backend
        self.c = c
        self.order = order
        self.wsafe = wsafe
        self.pairs = None  # [count] to tally treecode pair evaluations
        if backend == "tree":
            self.tree = Tree(self.x, max_depth=max_depth, leaf_cap=leaf_cap)
        elif backend == "direct":
            self._direct = direct
        elif backend == "numpy":
            from . import direct_np
            self._np = direct_np
        else:
            raise ValueError(backend)

    def __call__(self, op, nu, w):
        if self.backend == "tree":
            if self.pairs is not None:
                out, _, k = self.tree.apply(op, nu, w, self.c, order=self.order,
                                            wsafe=self.wsafe, with_stats=True)
                self.pairs[0] += int(k.sum())
                return out
            return self.tree.apply(op, nu, w, self.c, order=self.order, wsafe=self.wsafe)
        if self.backend == "direct":
            return self._direct(op, self.x, nu, w)
        return getattr(self._np, op)(self.x, nu, w)


def grad_step(ops, mu, w, b=0.5):
    """Alg. 2 for ||A_w mu - b||^2; returns (mu_new, alpha, r, E) where E is
    the energy of the incoming mu."""
    s = ops("A", mu, w)
    rho = b - s
    r = ops("AT", rho, w)
    t = ops("A", r, w)
    den = float((t * t).sum())
    alpha = float((r * r).sum()) / den if den > 0 else 0.0
    return mu + alpha * r, alpha, r, float((rho * rho).sum())


def orient(x, iters=40, w1=0.002, w2=0.016, mu0=None, backend="tree", c=2.0,
           max_depth=15, leaf_cap=1, start_iter=1, grad=True, wnnc=True,
           do_rescale=True, callback=None, schedule="linear", areas=None, order=0,
           wsafe=False, pair_count=None, timing=None):
    """Alg. 3 on normalized points x (n,3).  Returns mu (n,3) in FP64.

    grad / wnnc / do_rescale switch the three steps off for the ablations of
    Sec. 5.5 (defaults: the full method).  schedule and areas select the
    variants of the module docstring; order and wsafe the treecode's
    far-field extension (Tree.apply).  callback(i, mu, info) is called after
    every iteration.  pair_count (a list [n]) receives the number of treecode
    pair evaluations, timing (a dict) the seconds spent building the operators
    ("pre") and iterating ("main"): instrumentation only.
    """
    import time
    t0 = time.perf_counter()
    x = np.asarray(x, dtype=np.float64)
    ops = _Ops(x, backend, c, max_depth, leaf_cap, order, wsafe)
    ops.pairs = pair_count
    t1 = time.perf_counter()
    mu = np.zeros_like(x) if mu0 is None else np.array(mu0, dtype=np.float64)
    for i in range(start_iter, iters + 1):
        w = width_schedule(i, iters, w1, w2, schedule)
        info = {"w": w}
        if grad:
            mu, alpha, _, E = grad_step(ops, mu, w)
            info.update(alpha=alpha, E=E)
        if wnnc:
            mu_hat = ops("G", mu, w)
            mu = rescale(mu, mu_hat, areas) if do_rescale else mu_hat
        if callback is not None:
            callback(i, mu, info)
    if timing is not None:
        timing["pre"] = t1 - t0
        timing["main"] = time.perf_counter() - t1
    return mu
