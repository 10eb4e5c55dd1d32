"""kNN local-area estimate in FP64 -- TEST INFRASTRUCTURE ONLY.

The paper compares the solved areas |mu_i| with areas estimated from the k
nearest neighbours of each point, following Barill et al. 2018 (Sec. 6.1.2,
Table 5), and tests a rescale that enforces such areas (Sec. 6.1.1).  It gives
no formula; the reading implemented here:

1. the k nearest other points of the cloud (k = 16, fewer when the cloud is
   smaller; a point with fewer than 2 neighbours gets area 0);
2. the tangent plane's normal n: the eigenvector of the smallest eigenvalue of
   the covariance of the point and its neighbours about their mean;
3. an in-plane basis: e1 = the nearest neighbour's offset projected onto the
   plane and normalized (the next neighbour if that projection is 0),
   e2 = n x e1;
4. the neighbours' offsets projected to 2-D, u_j = (q_j . e1, q_j . e2);
5. the area of the Voronoi cell of the origin among the u_j (the intersection
   of the half-planes z . u_j <= |u_j|^2 / 2 over the u_j != 0), intersected
   with the square [-R, R]^2, R = max_j |u_j|, which bounds the cell of a
   point at the edge of an open surface.

On the 163,842-vertex unit icosphere this reading reproduces every printed
value of Table 5's kNN column (pinned in tests/test_oracle_pins.py).

Steps 1 and 5 use library primitives: a k-d tree query, and the half-plane
intersection and convex hull of Qhull (scipy.spatial).
"""
from __future__ import annotations

import numpy as np


def knn(x, k: int = 16):
    """Indices (n, min(k, n-1)) of the nearest other points, nearest first."""
    from scipy.spatial import cKDTree
    x = np.asarray(x, dtype=np.float64)
    m = min(k, len(x) - 1)
    if m < 1:
        return np.zeros((len(x), 0), np.int64)
    _, idx = cKDTree(x).query(x, m + 1)
    idx = np.asarray(idx).reshape(len(x), m + 1)
    # drop the point itself (first unless a coincident point came first)
    out = np.empty((len(x), m), np.int64)
    for i in range(len(x)):
        row = [j for j in idx[i] if j != i]
        out[i] = row[:m]
    return out


def tangent_normal(p, q):
    """Step 2: unit normal of the least-squares plane of p and its
    neighbours q (m,3)."""
    pts = np.vstack([p[None, :], q])
    c = pts - pts.mean(axis=0)
    _, vecs = np.linalg.eigh(c.T @ c)
    return vecs[:, 0]


def cell_area(u):
    """Step 5: area of the origin's Voronoi cell among the 2-D points u (m,2),
    clipped to [-R, R]^2."""
    from scipy.spatial import ConvexHull, HalfspaceIntersection
    u = np.asarray(u, dtype=np.float64)
    d = np.linalg.norm(u, axis=1)
    u = u[d > 0]
    if len(u) == 0:
        return 0.0
    R = d.max()
    # Qhull's convention: rows (a, b) with a . z + b <= 0
    hs = [np.array([ux, uy, -(ux * ux + uy * uy) / 2.0]) for ux, uy in u]
    hs += [np.array([1.0, 0.0, -R]), np.array([-1.0, 0.0, -R]),
           np.array([0.0, 1.0, -R]), np.array([0.0, -1.0, -R])]
    cut = HalfspaceIntersection(np.array(hs), np.zeros(2))
    return float(ConvexHull(cut.intersections).volume)


def knn_areas(x, k: int = 16, rows=None, nbr=None):
    """Areas (len(rows),) of the points x (n,3) of one cloud, steps 1-5.
    rows: the points to estimate (default all); nbr: precomputed neighbour
    indices (n, m) nearest first (default: step 1)."""
    x = np.asarray(x, dtype=np.float64)
    if nbr is None:
        nbr = knn(x, k)
    rows = np.arange(len(x)) if rows is None else np.asarray(rows)
    out = np.zeros(len(rows))
    for o, i in enumerate(rows):
        q = x[nbr[i][nbr[i] >= 0][:k]] - x[i]
        if len(q) < 2:
            continue
        n = tangent_normal(x[i], x[i] + q)
        t = q - np.outer(q @ n, n)
        tl = np.linalg.norm(t, axis=1)
        if not np.any(tl > 0):
            continue
        e1 = t[np.argmax(tl > 0)] / tl[np.argmax(tl > 0)]
        e2 = np.cross(n, e1)
        out[o] = cell_area(np.stack([q @ e1, q @ e2], axis=1))
    return out
