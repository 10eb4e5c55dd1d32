"""Vectorized numpy FP64 direct sums for small N (test infrastructure only).

A second transcription of the operators, independent of the C file, used on
clouds of at most a few thousand points:

  A  (Sec. 4.3):  s_i  = sum_j gradPhi(x_i - x_j) . mu_j
  A^T (Alg. 2):   v_j  = sum_i rho_i gradPhi(x_i - x_j)
  G  (Sec. 4.2):  mu^_i = -sum_j HPhi(x_i - x_j) mu_j

with gradPhi(y) = -y/(4 pi |y|^3) (Thm. 1), HPhi(y) = -I/(4 pi |y|^3) +
3 y y^T / (4 pi |y|^5) (Sec. 4.2), and every term with |y| < w (or y = 0)
set to zero (Sec. 4.4).
"""
from __future__ import annotations

import numpy as np


def _geometry(x, targets, w):
    x = np.asarray(x, dtype=np.float64)
    t = x if targets is None else np.asarray(targets, dtype=np.float64)
    y = t[:, None, :] - x[None, :, :]          # y = target - source
    r = np.sqrt((y * y).sum(axis=2))
    keep = (r >= w) & (r > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv3 = np.where(keep, 1.0 / (4.0 * np.pi * r ** 3), 0.0)
        inv5 = np.where(keep, 1.0 / (4.0 * np.pi * r ** 5), 0.0)
    return y, inv3, inv5


def A(x, mu, w, targets=None):
    y, inv3, _ = _geometry(x, targets, w)
    mu = np.asarray(mu, dtype=np.float64)
    return -(np.einsum("ijk,jk->ij", y, mu) * inv3).sum(axis=1)


def AT(x, rho, w, targets=None):
    # target j collects rho_i gradPhi(x_i - x_j) = rho_i (x_j - x_i)/(4 pi r^3)
    y, inv3, _ = _geometry(x, targets, w)
    rho = np.asarray(rho, dtype=np.float64)
    return np.einsum("ijk,ij->ik", y, inv3 * rho[None, :])


def G(x, mu, w, targets=None):
    y, inv3, inv5 = _geometry(x, targets, w)
    mu = np.asarray(mu, dtype=np.float64)
    ym = np.einsum("ijk,jk->ij", y, mu)
    return (inv3[:, :, None] * mu[None, :, :]).sum(axis=1) - 3.0 * np.einsum("ij,ijk->ik", ym * inv5, y)
