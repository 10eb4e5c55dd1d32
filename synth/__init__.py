"""Seeded synthetic point clouds for the WNNC normal-orientation workloads.

This module only draws inputs: point positions, their ground-truth normals,
area weights and random initial vectors.  It holds none of the method's
arithmetic (no winding numbers, no kernels, no trees), so that both the FP64
oracle and the GPU library can consume the very same arrays.

Every generator takes an explicit seed and uses ``numpy.random.default_rng``
(PCG64), so a given (generator, seed, size) always yields identical arrays.

Workloads (stand-ins for the paper's scanned and benchmark models, which are
not available; the paper's inputs are 1e4..2.4e6 points, uniform or noisy,
Sec. 5):

* ``fibonacci_sphere``  -- a jittered Fibonacci lattice on the unit sphere,
  the sphere sanity case of Thm. 1.
* ``ellipsoid_union``   -- points uniform by area on the boundary of a union
  of random ellipsoids inside the unit cube, with optional Gaussian noise of
  a fraction of the bounding-box diagonal (the noise model of Sec. 5.2.5).
* ``torus_knot``        -- a (2,3) torus-knot tube with a 10:1 sampling
  density variation along the curve plus uniform outliers (non-uniform raw
  scans with outliers, Sec. 5.2.6).
* ``torus_chain``       -- fused tori in a row, a closed surface of genus
  ``count`` (the high-genus case of Sec. 5.2.3).
* ``batched_sizes``     -- the log-uniform cloud sizes of the batched case.
* ``icosphere``         -- vertices of a subdivided icosahedron projected on
  the unit sphere (163,842 vertices at level 7: the sphere of Table 5).
* ``random_unit``       -- i.i.d. uniformly random unit vectors.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Cloud",
    "fibonacci_sphere",
    "ellipsoid_union",
    "torus_knot",
    "torus_chain",
    "batched_sizes",
    "batched_clouds",
    "icosphere",
    "random_unit",
    "config",
]


@dataclass
class Cloud:
    """A synthetic cloud.

    points : (N, 3) float32, caller order.
    normals: (N, 3) float32 ground-truth outward unit normals (NaN rows for
             outliers, which have none).
    area   : total surface area of the generating surface (float, original
             frame), so that ``area / N`` is a mean area weight.
    mu0    : (N, 3) float32 random initial unit vectors, or None.
    meta   : free-form description of the recipe.
    """

    points: np.ndarray
    normals: np.ndarray
    area: float
    mu0: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.points.shape[0])


def random_unit(rng: np.random.Generator, n: int) -> np.ndarray:
    """n i.i.d. uniformly random unit vectors (normalized standard normals)."""
    v = rng.standard_normal((n, 3))
    nrm = np.linalg.norm(v, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    return v / nrm


def fibonacci_sphere(n: int = 2000, seed: int = 0, jitter: float = 1e-3,
                     with_init: bool = True) -> Cloud:
    """Jittered Fibonacci lattice on the unit sphere.

    z_k = 1 - (2k+1)/n, phi_k = k*pi*(3 - sqrt 5).  Gaussian jitter with
    standard deviation ``jitter`` per axis is drawn first, the random initial
    unit vectors second.  Ground-truth normals are the clean lattice points.
    """
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    phi = k * np.pi * (3.0 - np.sqrt(5.0))
    rad = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    clean = np.stack([rad * np.cos(phi), rad * np.sin(phi), z], axis=1)
    rng = np.random.default_rng(seed)
    pts = clean + (rng.standard_normal((n, 3)) * jitter if jitter > 0 else 0.0)
    mu0 = random_unit(rng, n).astype(np.float32) if with_init else None
    return Cloud(points=pts.astype(np.float32), normals=clean.astype(np.float32),
                 area=4.0 * np.pi, mu0=mu0,
                 meta=dict(kind="fibonacci_sphere", n=n, seed=seed, jitter=jitter))


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a normalized Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([
        [a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
        [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
        [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d],
    ])


def _ellipsoid_area_mc(rng, axes, m=20000):
    u = random_unit(rng, m)
    jac = np.prod(axes) * np.linalg.norm(u / axes, axis=1)
    return 4.0 * np.pi * float(jac.mean())


def _sample_ellipsoid(rng, axes, count):
    """``count`` points uniform by area on the ellipsoid with semi-axes
    ``axes`` (local frame), with their outward unit normals."""
    out_p, out_n = [], []
    have = 0
    gmax = 1.0 / axes.min()
    while have < count:
        m = max(64, int(1.6 * (count - have)) + 64)
        u = random_unit(rng, m)
        g = np.linalg.norm(u / axes, axis=1)
        keep = rng.random(m) * gmax < g
        u = u[keep]
        p = u * axes
        nrm = u / axes
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        out_p.append(p)
        out_n.append(nrm)
        have += len(p)
    return np.concatenate(out_p)[:count], np.concatenate(out_n)[:count]


def ellipsoid_union(n: int = 50000, seed: int = 2, members: int = 6,
                    axis_range=(0.1, 0.4), noise: float = 0.0025,
                    with_init: bool = True) -> Cloud:
    """Points uniform by area on the boundary of a union of random ellipsoids.

    Each member has semi-axes ~ U[axis_range]^3, a uniform random rotation and
    a centre drawn uniformly such that its axis-aligned bounding box lies in
    [0,1]^3.  Every member is sampled with the same density per unit area and
    points that fall inside another member are discarded, which leaves points
    uniform by area on the union's boundary; a seeded subset of exactly ``n``
    is kept.  Ground truth is the owning member's outward normal.  Isotropic
    Gaussian noise with per-axis standard deviation ``noise`` times the
    bounding-box diagonal of the clean samples is added last.
    """
    rng = np.random.default_rng(seed)
    ell = []
    for _ in range(members):
        axes = rng.uniform(axis_range[0], axis_range[1], size=3)
        R = _random_rotation(rng)
        half = np.sqrt(((R * axes[None, :]) ** 2).sum(axis=1))
        ctr = rng.uniform(half, 1.0 - half)
        ell.append((axes, R, ctr))
    areas = np.array([_ellipsoid_area_mc(rng, a) for a, _, _ in ell])

    def inside_other(p, k):
        mask = np.zeros(len(p), dtype=bool)
        for j, (a, R, c) in enumerate(ell):
            if j == k:
                continue
            loc = (p - c) @ R  # rotate into member j's frame
            mask |= ((loc / a) ** 2).sum(axis=1) < 1.0
        return mask

    pts, nrms = [], []
    total = 0
    scale = 1.3
    while total < n:
        want = scale * (n - total) + 256
        for k, (a, R, c) in enumerate(ell):
            cnt = int(np.ceil(want * areas[k] / areas.sum()))
            p, nn = _sample_ellipsoid(rng, a, cnt)
            p = p @ R.T + c
            nn = nn @ R.T
            keep = ~inside_other(p, k)
            pts.append(p[keep])
            nrms.append(nn[keep])
            total += int(keep.sum())
        scale *= 1.5
    P = np.concatenate(pts)
    Nn = np.concatenate(nrms)
    sel = rng.choice(len(P), size=n, replace=False)
    P, Nn = P[sel], Nn[sel]
    # visible-surface area estimate: total member area times the kept fraction
    # is not tracked exactly; the mean member-area density is good enough for
    # an area weight of the right scale.
    diag = float(np.linalg.norm(P.max(axis=0) - P.min(axis=0)))
    if noise > 0:
        P = P + rng.standard_normal(P.shape) * (noise * diag)
    mu0 = random_unit(rng, n).astype(np.float32) if with_init else None
    return Cloud(points=P.astype(np.float32), normals=Nn.astype(np.float32),
                 area=float(areas.sum()), mu0=mu0,
                 meta=dict(kind="ellipsoid_union", n=n, seed=seed, members=members,
                           noise=noise, diag=diag))


def torus_chain(n: int = 8000, seed: int = 6, count: int = 6, R: float = 0.1,
                r: float = 0.025, spacing: float = 1.8, with_init: bool = True) -> Cloud:
    """A closed surface of genus ``count``: ``count`` equal tori (major radius
    R, tube radius r, axis z) with centres on a line ``spacing * R`` apart,
    so that neighbouring tubes fuse while every hole stays open (the
    high-genus case of Sec. 5.2.3).  Each torus is sampled uniformly by
    area (u, v uniform, v accepted with probability (R + r cos v)/(R + r));
    points inside another torus are discarded and a seeded subset of exactly
    ``n`` is kept.  Ground truth is the owning torus's outward normal.  The
    chain is centred in [0,1]^3.
    """
    rng = np.random.default_rng(seed)
    cx = (np.arange(count) - (count - 1) / 2.0) * spacing * R + 0.5

    def inside(p, k):
        mask = np.zeros(len(p), dtype=bool)
        for j in range(count):
            if j == k:
                continue
            rho = np.hypot(p[:, 0] - cx[j], p[:, 1] - 0.5)
            mask |= (rho - R) ** 2 + (p[:, 2] - 0.5) ** 2 < r * r
        return mask

    pts, nrms = [], []
    total = 0
    per = int(1.5 * n / count) + 64
    while total < n:
        for k in range(count):
            u = rng.uniform(0.0, 2.0 * np.pi, per)
            v = rng.uniform(0.0, 2.0 * np.pi, per)
            keep = rng.random(per) * (R + r) < R + r * np.cos(v)
            u, v = u[keep], v[keep]
            rho = R + r * np.cos(v)
            p = np.stack([cx[k] + rho * np.cos(u), 0.5 + rho * np.sin(u), 0.5 + r * np.sin(v)], 1)
            nn = np.stack([np.cos(v) * np.cos(u), np.cos(v) * np.sin(u), np.sin(v)], 1)
            ok = ~inside(p, k)
            pts.append(p[ok])
            nrms.append(nn[ok])
            total += int(ok.sum())
    P = np.concatenate(pts)
    Nn = np.concatenate(nrms)
    sel = rng.choice(len(P), size=n, replace=False)
    P, Nn = P[sel], Nn[sel]
    mu0 = random_unit(rng, n).astype(np.float32) if with_init else None
    return Cloud(points=P.astype(np.float32), normals=Nn.astype(np.float32),
                 area=float(count * 4 * np.pi ** 2 * R * r), mu0=mu0,
                 meta=dict(kind="torus_chain", n=n, seed=seed, count=count, R=R, r=r,
                           spacing=spacing))


def _rmf(curve_pts, tangents):
    """Rotation-minimizing frame by the double-reflection method
    (Wang, Juttler, Zheng, Liu 2008)."""
    m = len(curve_pts)
    t0 = tangents[0]
    a = np.array([1.0, 0.0, 0.0]) if abs(t0[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    r = np.cross(t0, a)
    r /= np.linalg.norm(r)
    R = np.empty((m, 3))
    R[0] = r
    for i in range(m - 1):
        v1 = curve_pts[i + 1] - curve_pts[i]
        c1 = v1 @ v1
        rL = r - (2.0 / c1) * (v1 @ r) * v1
        tL = tangents[i] - (2.0 / c1) * (v1 @ tangents[i]) * v1
        v2 = tangents[i + 1] - tL
        c2 = v2 @ v2
        r = rL - (2.0 / c2) * (v2 @ rL) * v2 if c2 > 0 else rL
        r /= np.linalg.norm(r)
        R[i + 1] = r
    return R


def torus_knot(n: int = 500000, seed: int = 3, outlier_frac: float = 0.02,
               p: int = 2, q: int = 3, R: float = 0.3, r: float = 0.12,
               tube: float = 0.05, density_ratio: float = 10.0,
               with_init: bool = True, samples: int = 20000) -> Cloud:
    """A (p,q) torus-knot tube with sampling density varying along the curve.

    Centreline (1/2,1/2,1/2) + ((R + r cos qt) cos pt, (R + r cos qt) sin pt,
    r sin qt).  The tube of radius ``tube`` is swept with a rotation-minimizing
    frame; points are drawn with density proportional to the tube's area
    element times g(s) = 1 + (density_ratio-1)(1 + cos(2 pi s/L))/2 along the
    arc length s, so the densest and sparsest parts differ by density_ratio.
    A fraction ``outlier_frac`` of the n points are uniform outliers in the
    surface points' bounding box (normals NaN).
    """
    rng = np.random.default_rng(seed)
    n_out = int(round(n * outlier_frac))
    n_surf = n - n_out
    t = np.linspace(0.0, 2.0 * np.pi, samples, endpoint=False)

    def curve(tt):
        rr = R + r * np.cos(q * tt)
        return np.stack([rr * np.cos(p * tt), rr * np.sin(p * tt), r * np.sin(q * tt)], axis=1) + 0.5

    def dcurve(tt):
        rr = R + r * np.cos(q * tt)
        drr = -r * q * np.sin(q * tt)
        return np.stack([drr * np.cos(p * tt) - rr * p * np.sin(p * tt),
                         drr * np.sin(p * tt) + rr * p * np.cos(p * tt),
                         r * q * np.cos(q * tt)], axis=1)

    C = curve(t)
    D1 = dcurve(t)
    speed = np.linalg.norm(D1, axis=1)
    T = D1 / speed[:, None]
    dt = 2.0 * np.pi / samples
    s_cum = np.concatenate([[0.0], np.cumsum(speed * dt)])[:-1]
    L = float((speed * dt).sum())
    # curvature vector kappa*N = dT/ds (central differences on the closed curve)
    dT = (np.roll(T, -1, axis=0) - np.roll(T, 1, axis=0)) / (2.0 * dt)
    K = dT / speed[:, None]
    N1 = _rmf(C, T)
    N2 = np.cross(T, N1)
    g = 1.0 + (density_ratio - 1.0) * (1.0 + np.cos(2.0 * np.pi * s_cum / L)) / 2.0
    w_seg = speed * dt * g
    w_seg /= w_seg.sum()
    kmax = float(np.linalg.norm(K, axis=1).max())
    amax = 1.0 + tube * kmax
    pts, nrms = [], []
    have = 0
    while have < n_surf:
        m = int(1.4 * (n_surf - have)) + 1024
        idx = rng.choice(samples, size=m, p=w_seg)
        phi = rng.uniform(0.0, 2.0 * np.pi, size=m)
        e = np.cos(phi)[:, None] * N1[idx] + np.sin(phi)[:, None] * N2[idx]
        jac = 1.0 - tube * (e * K[idx]).sum(axis=1)
        keep = rng.random(m) * amax < jac
        pts.append(C[idx][keep] + tube * e[keep])
        nrms.append(e[keep])
        have += int(keep.sum())
    P = np.concatenate(pts)[:n_surf]
    Nn = np.concatenate(nrms)[:n_surf]
    lo, hi = P.min(axis=0), P.max(axis=0)
    O = rng.uniform(lo, hi, size=(n_out, 3))
    P = np.concatenate([P, O])
    Nn = np.concatenate([Nn, np.full((n_out, 3), np.nan)])
    mu0 = random_unit(rng, n).astype(np.float32) if with_init else None
    area = 2.0 * np.pi * tube * L
    return Cloud(points=P.astype(np.float32), normals=Nn.astype(np.float32),
                 area=area, mu0=mu0,
                 meta=dict(kind="torus_knot", n=n, seed=seed, p=p, q=q, tube=tube,
                           outliers=n_out, density_ratio=density_ratio, length=L))


def batched_sizes(count: int = 64, seed: int = 1, lo: float = 5e3, hi: float = 2e5) -> np.ndarray:
    """Cloud sizes floor(exp(U[ln lo, ln hi])) drawn first from rng(seed)."""
    rng = np.random.default_rng(seed)
    return np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)


def batched_clouds(count: int = 64, seed: int = 1, sizes=None):
    """``count`` noise-free ellipsoid unions with log-uniform sizes; cloud k
    uses seed 1000*seed + k."""
    if sizes is None:
        sizes = batched_sizes(count, seed)
    return [ellipsoid_union(int(m), seed=1000 * seed + k, noise=0.0, with_init=False)
            for k, m in enumerate(sizes)]


def icosphere(level: int = 7) -> Cloud:
    """Vertices of an icosahedron subdivided ``level`` times (each triangle
    split into four, new vertices projected to the unit sphere).  Level 7 has
    10*4^7 + 2 = 163,842 vertices."""
    t = (1.0 + np.sqrt(5.0)) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = np.array(V, dtype=np.float64)
    verts /= np.linalg.norm(verts, axis=1, keepdims=True)
    faces = np.array(F, dtype=np.int64)
    for _ in range(level):
        e = np.concatenate([faces[:, [0, 1]], faces[:, [1, 2]], faces[:, [2, 0]]])
        e.sort(axis=1)
        uniq, inv = np.unique(e, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mid = verts[uniq[:, 0]] + verts[uniq[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = len(verts)
        verts = np.concatenate([verts, mid])
        nf = len(faces)
        a = base + inv[:nf]
        b = base + inv[nf:2 * nf]
        c = base + inv[2 * nf:]
        f0, f1, f2 = faces[:, 0], faces[:, 1], faces[:, 2]
        faces = np.concatenate([
            np.stack([f0, a, c], axis=1), np.stack([f1, b, a], axis=1),
            np.stack([f2, c, b], axis=1), np.stack([a, b, c], axis=1)])
    return Cloud(points=verts.astype(np.float32), normals=verts.astype(np.float32),
                 area=4.0 * np.pi, mu0=None,
                 meta=dict(kind="icosphere", level=level, n=len(verts), faces=faces))


def config(name: str) -> dict:
    """The workloads with their method settings (widths in the normalized
    frame, iteration count, treecode threshold c and depth D).

    The defaults of Sec. 5.1: w1 = 0.002, w2 = 0.016, c = 2, D = 15, 40
    iterations; the noisy case uses the 0.25 % noise widths w1 = 0.02,
    w2 = 4 w1 of Sec. 5.2.5.
    """
    if name == "sphere2k":
        return dict(make=lambda: fibonacci_sphere(2000, 0), w1=0.002, w2=0.016,
                    iters=40, c=2.0, depth=15)
    if name == "ellipsoids50k":
        return dict(make=lambda: ellipsoid_union(50000, 2), w1=0.02, w2=0.08,
                    iters=40, c=2.0, depth=15)
    if name == "torusknot500k":
        return dict(make=lambda: torus_knot(500000, 3), w1=0.002, w2=0.016,
                    iters=40, c=2.0, depth=15)
    raise KeyError(name)
