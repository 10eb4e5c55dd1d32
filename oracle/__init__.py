"""FP64 CPU oracle for WNNC normal orientation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
and never imports it.

Contents (paper: Lin, Shi, Liu 2024, WNNC normal orientation):

* ``normalize``            -- the input normalization of Sec. 5.1.1.
* ``direct``               -- exact O(N^2) FP64 sums of A, A^T, G with the
                              smoothing cutoff (Thm. 1, Sec. 4.2, Sec. 4.4),
                              in C (``liboracle.so``).
* ``direct_np``            -- the same sums in vectorized numpy for small N
                              (a second, independent transcription).
* ``Tree``                 -- the paper's treecode (Sec. 4.5, Alg. 4) in C.
* ``grad_step``/``orient`` -- Alg. 2 and Alg. 3 (``iterate.py``), with the
                              width-schedule and fixed-area variants.
* ``areas.knn_areas``      -- the kNN local-area estimate of Sec. 6.1 and
                              Table 5 (``areas.py``).

Parity pins: see the module docstrings of ``direct_np`` and ``iterate`` and
the ``tests/test_oracle_*.py`` files.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

OP_A, OP_AT, OP_G, OP_P, OP_T = 0, 1, 2, 3, 4
_OPS = {"A": OP_A, "AT": OP_AT, "G": OP_G, "P": OP_P, "T": OP_T}
_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # WNNC_ORACLE_LIB: another build of the same source (the sanitizer test)
    path = os.environ.get("WNNC_ORACLE_LIB") or _build.build(force=False)
    lib = ctypes.CDLL(path)
    d = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.or_direct.argtypes = [ctypes.c_int, d, i64, d, d, i64, ctypes.c_double, d, d]
    lib.or_direct.restype = None
    lib.or_direct_tv.argtypes = [ctypes.c_int, d, i64, d, d, i64, d, ctypes.c_double, d, d]
    lib.or_direct_tv.restype = None
    lib.or_tree_new.argtypes = [d, i64, ctypes.c_int, ctypes.c_int]
    lib.or_tree_new.restype = ctypes.c_void_p
    lib.or_tree_free.argtypes = [ctypes.c_void_p]
    lib.or_tree_nnodes.argtypes = [ctypes.c_void_p]
    lib.or_tree_nnodes.restype = i64
    p32 = ctypes.POINTER(ctypes.c_int32)
    p64 = ctypes.POINTER(ctypes.c_int64)
    lib.or_tree_export.argtypes = [ctypes.c_void_p, p32, p32, p64, p64, p64]
    lib.or_tree_reps.argtypes = [ctypes.c_void_p, d, ctypes.c_int, d, d, d]
    lib.or_tree_apply.argtypes = [ctypes.c_void_p, ctypes.c_int, d, ctypes.c_double,
                                  ctypes.c_double, d, i64, d, d, p64]
    lib.or_tree_apply_tv.argtypes = [ctypes.c_void_p, ctypes.c_int, d, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_int, d, i64, d, d,
                                     d, p64]
    lib.or_tree_apply_margins.argtypes = [ctypes.c_void_p, ctypes.c_int, d, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_int, ctypes.c_int, d, i64, d,
                                          d, d, p64, d]
    lib.or_tree_apply_order.argtypes = [ctypes.c_void_p, ctypes.c_int, d, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, ctypes.c_int, d, i64, d,
                                        d, p64]
    lib.or_num_threads.restype = ctypes.c_int
    lib.or_set_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_threads(n: int) -> None:
    _load().or_set_threads(int(n))


def normalize(points):
    """Sec. 5.1.1: fit the cloud into [-1,1]^3 with a margin of 1/11.

    Reading: centre = midpoint of the bounding box; one uniform scale so that
    the largest half-extent becomes 1 - 1/11 = 10/11.  Computed in FP64 from
    the FP32 input and rounded once to FP32.  Returns (x32, center, scale)
    with x = (p - center) * scale.
    """
    p = np.asarray(points, dtype=np.float32).astype(np.float64)
    lo = p.min(axis=0)
    hi = p.max(axis=0)
    center = (lo + hi) / 2.0
    half = float(((hi - lo) / 2.0).max())
    scale = (10.0 / 11.0) / half if half > 0 else 1.0
    x = ((p - center) * scale).astype(np.float32)
    return x, center, scale


def direct(op: str, x, nu, w: float, targets=None, with_mag: bool = False, tvec=None):
    """Exact FP64 sum of operator op in {"A","AT","G","P","T"} over all source
    points x (n,3) with attributes nu ((n,3) for A, G and T, (n,) for AT and
    P), evaluated at targets (default: the points themselves); P and T also
    take the targets' vectors tvec (n_targets,3)."""
    lib = _load()
    o = _OPS[op]
    x = _f64(x, (-1, 3))
    nu = _f64(nu, (x.shape[0], -1) if o not in (OP_AT, OP_P) else (x.shape[0],))
    t = x if targets is None else _f64(targets, (-1, 3))
    dout = 1 if o == OP_A else 3
    out = np.zeros((t.shape[0], dout))
    mag = np.zeros(t.shape[0])
    tv = _tvec(o, tvec, t.shape[0])
    lib.or_direct_tv(o, _dp(x), x.shape[0], _dp(nu), _dp(t), t.shape[0],
                     _dp(tv) if tv is not None else None, float(w), _dp(out), _dp(mag))
    out = out[:, 0] if dout == 1 else out
    return (out, mag) if with_mag else out


def _tvec(o, tvec, n):
    if o not in (OP_P, OP_T):
        return None
    if tvec is None:
        raise ValueError("P needs the targets' vectors")
    return _f64(tvec, (n, 3))


class Tree:
    """The paper's octree and treecode (Sec. 4.5, Alg. 4), FP64, in C."""

    def __init__(self, x, max_depth: int = 15, leaf_cap: int = 1):
        lib = _load()
        self.x = _f64(x, (-1, 3))
        self.n = self.x.shape[0]
        self.max_depth = int(max_depth)
        self.leaf_cap = int(leaf_cap)
        self._h = lib.or_tree_new(_dp(self.x), self.n, self.max_depth, self.leaf_cap)
        if not self._h:
            raise ValueError("invalid tree parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_tree_free(h)
            self._h = None

    @property
    def nnodes(self) -> int:
        return int(_load().or_tree_nnodes(self._h))

    def export(self):
        """(depth, leaf, begin, end, order): node member sets are
        order[begin[k]:end[k]] (caller indices)."""
        m = self.nnodes
        depth = np.zeros(m, np.int32)
        leaf = np.zeros(m, np.int32)
        begin = np.zeros(m, np.int64)
        end = np.zeros(m, np.int64)
        order = np.zeros(self.n, np.int64)
        P32 = ctypes.POINTER(ctypes.c_int32)
        P64 = ctypes.POINTER(ctypes.c_int64)
        _load().or_tree_export(self._h, depth.ctypes.data_as(P32), leaf.ctypes.data_as(P32),
                               begin.ctypes.data_as(P64), end.ctypes.data_as(P64),
                               order.ctypes.data_as(P64))
        return depth, leaf, begin, end, order

    def reps(self, nu):
        """nu-representatives of every node: (x_B (m,3), nu_B (m,3|1), W (m,))."""
        nu = np.asarray(nu, dtype=np.float64)
        dim = 1 if nu.ndim == 1 else 3
        nu = _f64(nu, (self.n, dim))
        m = self.nnodes
        xB = np.zeros((m, 3))
        nuB = np.zeros((m, 3))
        W = np.zeros(m)
        _load().or_tree_reps(self._h, _dp(nu), dim, _dp(xB), _dp(nuB), _dp(W))
        return xB, (nuB[:, 0] if dim == 1 else nuB), W

    def apply(self, op: str, nu, w: float, c: float = 2.0, targets=None, with_stats: bool = False,
              order: int = 0, wsafe: bool = False, tvec=None, with_margins: bool = False):
        """Treecode operator; returns out (and per-target magnitude sums and
        pair counts with with_stats).  order 1 or 2 replaces each accepted
        node's representative term by the Taylor expansion of the pair term
        about x_B to that order (the higher-order far field; 0 is Alg. 4).

        with_margins appends, per target, the decision margins (n_targets, 2):
        column 0 the smallest |dist - thr| / thr over the acceptance tests of
        Alg. 4 it evaluated, column 1 the smallest |r - w| / w over the pair
        terms it formed (the cutoff of Sec. 4.4; inf for w = 0).  Diagnostics
        only: the result does not depend on them."""
        lib = _load()
        o = _OPS[op]
        nu = _f64(nu, (self.n, 3) if o not in (OP_AT, OP_P) else (self.n,))
        t = self.x if targets is None else _f64(targets, (-1, 3))
        if o in (OP_P, OP_T) and order != 0:
            raise ValueError("P and T have the representative far field only")
        tv = _tvec(o, tvec, t.shape[0])
        dout = 1 if o == OP_A else 3
        out = np.zeros((t.shape[0], dout))
        mag = np.zeros(t.shape[0])
        pairs = np.zeros(t.shape[0], np.int64)
        if order not in (0, 1, 2):
            raise ValueError("order must be 0, 1 or 2")
        margins = np.zeros((t.shape[0], 2)) if with_margins else None
        lib.or_tree_apply_margins(self._h, o, _dp(nu), float(w), float(c), int(order),
                                  int(bool(wsafe)), _dp(t), t.shape[0],
                                  _dp(tv) if tv is not None else None, _dp(out), _dp(mag),
                                  pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  _dp(margins) if margins is not None else None)
        out = out[:, 0] if dout == 1 else out
        res = (out, mag, pairs) if with_stats else (out,)
        if with_margins:
            res = res + (margins,)
        return res if len(res) > 1 else res[0]


def winding_grad_x(x, mu, g, w: float, backend: str = "direct", c: float = 2.0, tree=None):
    """Gradient with respect to the points x of L = sum_i g_i s_i, s = A_w(mu)
    (an extension: differentiable winding numbers in the positions).  With
    s_i = sum_j gradPhi(x_i - x_j) . mu_j, differentiating each pair term in
    both of its end points gives
      dL/dx_k = g_k sum_j HPhi(x_k - x_j) mu_j - sum_i g_i HPhi(x_i - x_k) mu_k
              = -g_k G(mu)_k + P(g; mu)_k
    (HPhi is even).  Pairs cut off at w contribute nothing (the cutoff is
    held fixed).  backend "direct" (exact sums) or "tree" (the treecode, both
    terms with Alg. 4's far field)."""
    x = np.asarray(x, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    if backend == "direct":
        G = direct("G", x, mu, w)
        P = direct("P", x, g, w, tvec=mu)
    else:
        T = tree if tree is not None else Tree(x)
        G = T.apply("G", mu, w, c)
        P = T.apply("P", g, w, c, tvec=mu)
    return -g[:, None] * G + P


def gradient_grad_x(x, mu, v, w: float, backend: str = "direct", c: float = 2.0, tree=None):
    """Gradient with respect to the points x of L = sum_i v_i . grad F(x_i; mu)
    (grad F = -G(mu); an extension).  With grad F_i = sum_j HPhi(x_i - x_j) mu_j,
    differentiating each pair term in both end points (T3Phi odd) gives
      dL/dx_k = sum_j T3Phi(x_k - x_j)[v_k, mu_j] + sum_i T3Phi(x_k - x_i)[mu_k, v_i]
              = T(mu; v)_k + T(v; mu)_k
    (T(a; b): sources a, target vectors b).  The cutoff is held fixed."""
    x = np.asarray(x, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    if backend == "direct":
        return direct("T", x, mu, w, tvec=v) + direct("T", x, v, w, tvec=mu)
    T = tree if tree is not None else Tree(x)
    return T.apply("T", mu, w, c, tvec=v) + T.apply("T", v, w, c, tvec=mu)


from .iterate import grad_step, orient, width_schedule, rescale  # noqa: E402
from . import direct_np  # noqa: E402,F401
