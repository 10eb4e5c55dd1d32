"""Normal-quality metrics of Sec. 5.1.4 (host side, numpy; not part of the
device path).

* AE_pcd = mean over points of (1 - n_gt . n) / 2, unit normals;
* P_co   = fraction of points with n . n_gt > 0 (correctly oriented);
* flip rate between two results = fraction with a . b <= 0.

Points without a reference normal (non-finite rows of n_gt, such as the
outliers of the synthetic scans) and zero vectors are left out, and so are
rows outside an optional boolean mask.
"""
from __future__ import annotations

import numpy as np


def _rows(a, b, mask=None):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    na = np.linalg.norm(a, axis=1)
    nb = np.linalg.norm(b, axis=1)
    ok = np.isfinite(na) & np.isfinite(nb) & (na > 0) & (nb > 0)
    if mask is not None:
        ok &= np.asarray(mask, dtype=bool)
    cos = (a[ok] * b[ok]).sum(axis=1) / (na[ok] * nb[ok])
    return cos


def ae_pcd(n, n_gt, mask=None) -> float:
    """Mean angular error (1 - cos)/2 of the directions n against n_gt."""
    cos = _rows(n, n_gt, mask)
    return float(((1.0 - cos) / 2.0).mean()) if cos.size else float("nan")


def p_co(n, n_gt, mask=None) -> float:
    """Fraction of correctly oriented normals (n . n_gt > 0)."""
    cos = _rows(n, n_gt, mask)
    return float((cos > 0).mean()) if cos.size else float("nan")


def flip_rate(a, b, mask=None) -> float:
    """Fraction of rows whose directions disagree (a . b <= 0)."""
    cos = _rows(a, b, mask)
    return float((cos <= 0).mean()) if cos.size else float("nan")
