"""Python binding of the MI355X WNNC library (libwnnc.so, C ABI in include/wnnc.h).

The functions named ``wnnc_*`` mirror the C entry points one to one and only
marshal arguments: torch CUDA tensors are passed as device pointers and the
current torch stream is used unless a stream is given.  Every computation runs
in the library's HIP kernels; there is no fallback.  If the shared library has
not been built, importing the binding raises with the command to build it.

``Context`` wraps a context handle for convenience; ``autograd`` holds the
differentiable winding-number functions.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwnnc.so")

WNNC_OK, WNNC_EINVAL, WNNC_ENOMEM, WNNC_EDEVICE, WNNC_ESTATE, WNNC_ENUMERIC = 0, -1, -2, -3, -4, -5
FLAG_COUNT_PAIRS = 1
FLAG_TIME_KERNELS = 2
FLAG_CHECK_FINITE = 4
FLAG_TIME_TRAVERSAL = 8
FLAG_SEPARATE_COMBINE = 16
OP_A, OP_AT, OP_G = 0, 1, 2

EXPORTED = [
    "wnnc_create", "wnnc_destroy", "wnnc_set_stream", "wnnc_set_flags", "wnnc_normalize",
    "wnnc_build", "wnnc_winding", "wnnc_gradient", "wnnc_adjoint", "wnnc_orient",
    "wnnc_orient_energy", "wnnc_stats", "wnnc_reset_stats", "wnnc_tree_export",
    "wnnc_moments_export", "wnnc_normals", "wnnc_last_error", "wnnc_version",
    "wnnc_normalize_batched", "wnnc_build_batched", "wnnc_set_tile", "wnnc_get_tile",
    "wnnc_autotune", "wnnc_orient_preset", "wnnc_knn_features", "wnnc_knn_areas",
    "wnnc_mlp_forward", "wnnc_mlp_grad", "wnnc_mlp_adam",
    "wnnc_warm_orient", "wnnc_set_prefetch", "wnnc_set_split", "wnnc_get_split",
    "wnnc_winding_at", "wnnc_set_far_field", "wnnc_get_far_field", "wnnc_winding_grad_x",
    "wnnc_gradient_grad_x", "wnnc_energy", "wnnc_winding_grad_x_noalloc", "wnnc_set_defer",
    "wnnc_get_defer",
]
NOALLOC_MAX_POINTS = 1 << 20
MLP_PARAMS = 7491
AUTOTUNE_CONFIGS = 16
MAX_SPLIT = 1 << 20


class WnncError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"wnnc status {status}: {msg}")
        self.status = status


class TreeOpts(ctypes.Structure):
    _fields_ = [("c", ctypes.c_float), ("max_depth", ctypes.c_int), ("leaf_cap", ctypes.c_int)]


class OrientOpts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("w1", ctypes.c_float), ("w2", ctypes.c_float),
                ("start_iter", ctypes.c_int), ("stop_iter", ctypes.c_int),
                ("schedule", ctypes.c_int), ("areas", ctypes.c_void_p)]


SCHEDULES = {"linear": 0, "cosine": 1, "exponential": 2}
PRESETS = {"default": 0, "noise_0.25": 1, "noise_0.5": 2, "noise_1": 3, "scan": 4,
           "high_genus": 5}


class WarmOpts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("w1", ctypes.c_float), ("w2", ctypes.c_float),
                ("max_disagree", ctypes.c_float), ("fallback_iters", ctypes.c_int),
                ("fallback_w2", ctypes.c_float), ("max_pred_disagree", ctypes.c_float),
                ("max_iters", ctypes.c_int), ("stop_frac", ctypes.c_float)]


class WarmReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("fallback", ctypes.c_int),
                ("max_disagree", ctypes.c_double), ("max_pred_disagree", ctypes.c_double)]


class TileTime(ctypes.Structure):
    _fields_ = [("tpl", ctypes.c_int), ("prefetch", ctypes.c_int), ("split", ctypes.c_int),
                ("ms", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("calls", ctypes.c_int64 * 5), ("pairs", ctypes.c_int64 * 5),
                ("traverse_ms", ctypes.c_double * 5), ("moments_ms", ctypes.c_double),
                ("build_ms", ctypes.c_double), ("n_clouds", ctypes.c_int64),
                ("tile", ctypes.c_int64), ("n_groups", ctypes.c_int64),
                ("n_tasks", ctypes.c_int64), ("combine_ms", ctypes.c_double),
                ("prefetch_ops", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return dict(n_points=self.n_points, n_nodes=self.n_nodes, calls=list(self.calls),
                    pairs=list(self.pairs), traverse_ms=list(self.traverse_ms),
                    moments_ms=self.moments_ms, build_ms=self.build_ms,
                    n_clouds=self.n_clouds, tile=self.tile, n_groups=self.n_groups,
                    n_tasks=self.n_tasks, combine_ms=self.combine_ms,
                    prefetch_ops=self.prefetch_ops)


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libwnnc.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing; build it with `python -m paper_2405_16634_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, f32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_float, ctypes.c_double
    P = ctypes.POINTER
    sigs = {
        "wnnc_create": [P(vp), ctypes.c_int, vp],
        "wnnc_destroy": [vp],
        "wnnc_set_stream": [vp, vp],
        "wnnc_set_flags": [vp, ctypes.c_uint],
        "wnnc_normalize": [vp, vp, i64, vp, P(dbl)],
        "wnnc_build": [vp, vp, i64, P(TreeOpts)],
        "wnnc_winding": [vp, vp, vp, f32, vp],
        "wnnc_winding_at": [vp, vp, vp, f32, vp, i64, vp],
        "wnnc_gradient": [vp, vp, vp, f32, vp],
        "wnnc_adjoint": [vp, vp, f32, vp],
        "wnnc_energy": [vp, vp, f32, dbl, P(dbl), vp],
        "wnnc_orient": [vp, P(OrientOpts), vp, vp],
        "wnnc_orient_energy": [vp, P(dbl), ctypes.c_int],
        "wnnc_stats": [vp, P(Stats)],
        "wnnc_reset_stats": [vp],
        "wnnc_tree_export": [vp, vp, vp, vp, vp, vp],
        "wnnc_moments_export": [vp, vp, ctypes.c_int, vp, vp, vp],
        "wnnc_normals": [vp, vp, i64, dbl, vp, vp],
        "wnnc_normalize_batched": [vp, vp, P(i64), ctypes.c_int, vp, P(dbl)],
        "wnnc_build_batched": [vp, vp, P(i64), ctypes.c_int, P(TreeOpts)],
        "wnnc_set_tile": [vp, ctypes.c_int],
        "wnnc_set_defer": [vp, ctypes.c_int],
        "wnnc_get_defer": [vp, P(ctypes.c_int)],
        "wnnc_get_tile": [vp, P(ctypes.c_int)],
        "wnnc_autotune": [vp, f32, P(TileTime)],
        "wnnc_set_prefetch": [vp, ctypes.c_int],
        "wnnc_set_split": [vp, ctypes.c_int],
        "wnnc_get_split": [vp, P(ctypes.c_int)],
        "wnnc_knn_features": [vp, vp, vp],
        "wnnc_knn_areas": [vp, ctypes.c_int, vp],
        "wnnc_orient_preset": [ctypes.c_int, P(OrientOpts)],
        "wnnc_set_far_field": [vp, ctypes.c_int, ctypes.c_int],
        "wnnc_winding_grad_x": [vp, vp, vp, f32, vp, vp],
        "wnnc_winding_grad_x_noalloc": [vp, vp, vp, f32, vp, vp],
        "wnnc_gradient_grad_x": [vp, vp, vp, f32, vp, vp],
        "wnnc_get_far_field": [vp, P(ctypes.c_int), P(ctypes.c_int)],
        "wnnc_mlp_forward": [vp, vp, vp, i64, vp],
        "wnnc_mlp_grad": [vp, vp, vp, vp, i64, vp, P(dbl)],
        "wnnc_mlp_adam": [vp, vp, vp, vp, vp, ctypes.c_int, f32, f32, f32, f32],
        "wnnc_warm_orient": [vp, vp, P(WarmOpts), vp, P(WarmReport)],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.wnnc_last_error.argtypes = []
    lib.wnnc_last_error.restype = ctypes.c_char_p
    lib.wnnc_version.argtypes = []
    lib.wnnc_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != WNNC_OK:
        msg = load_library().wnnc_last_error().decode(errors="replace")
        raise WnncError(status, msg)


def _dev(t, name, dtype=torch.float32, shape=None):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


# ------------------------------------------------------- C-ABI mirrors --

def wnnc_version() -> str:
    return load_library().wnnc_version().decode()


def wnnc_last_error() -> str:
    return load_library().wnnc_last_error().decode(errors="replace")


def wnnc_create(device: int = 0, stream=None):
    h = ctypes.c_void_p()
    _check(load_library().wnnc_create(ctypes.byref(h), int(device), _stream_ptr(stream)))
    return h


def wnnc_destroy(ctx) -> None:
    _check(load_library().wnnc_destroy(ctx))


def wnnc_set_stream(ctx, stream=None) -> None:
    _check(load_library().wnnc_set_stream(ctx, _stream_ptr(stream)))


def wnnc_set_flags(ctx, flags: int) -> None:
    _check(load_library().wnnc_set_flags(ctx, int(flags)))


def wnnc_normalize(ctx, P, P_norm):
    n = P.shape[0]
    cs = (ctypes.c_double * 4)()
    _check(load_library().wnnc_normalize(ctx, _dev(P, "P", shape=(n, 3)), n,
                                         _dev(P_norm, "P_norm", shape=(n, 3)), cs))
    return (cs[0], cs[1], cs[2]), cs[3]


def _offsets(offsets):
    arr = (ctypes.c_int64 * len(offsets))(*[int(v) for v in offsets])
    return arr, len(offsets) - 1


def wnnc_normalize_batched(ctx, P, P_norm, offsets):
    """Normalize each cloud (rows offsets[c]..offsets[c+1]) on its own.
    Returns a list of (centre, scale) per cloud."""
    n = P.shape[0]
    off, B = _offsets(offsets)
    cs = (ctypes.c_double * (4 * B))()
    _check(load_library().wnnc_normalize_batched(ctx, _dev(P, "P", shape=(n, 3)), off, B,
                                                 _dev(P_norm, "P_norm", shape=(n, 3)), cs))
    return [((cs[4 * k], cs[4 * k + 1], cs[4 * k + 2]), cs[4 * k + 3]) for k in range(B)]


def wnnc_build_batched(ctx, P, offsets, c: float = 2.0, max_depth: int = 15,
                       leaf_cap: int = 1) -> None:
    n = P.shape[0]
    off, B = _offsets(offsets)
    opts = TreeOpts(float(c), int(max_depth), int(leaf_cap))
    _check(load_library().wnnc_build_batched(ctx, _dev(P, "P", shape=(n, 3)), off, B,
                                             ctypes.byref(opts)))


def wnnc_set_tile(ctx, tpl: int) -> None:
    _check(load_library().wnnc_set_tile(ctx, int(tpl)))


def wnnc_get_tile(ctx) -> int:
    v = ctypes.c_int()
    _check(load_library().wnnc_get_tile(ctx, ctypes.byref(v)))
    return v.value


def wnnc_set_prefetch(ctx, on: bool) -> None:
    _check(load_library().wnnc_set_prefetch(ctx, 1 if on else 0))


def wnnc_set_split(ctx, visits: int) -> None:
    _check(load_library().wnnc_set_split(ctx, int(visits)))


def wnnc_get_split(ctx) -> int:
    v = ctypes.c_int()
    _check(load_library().wnnc_get_split(ctx, ctypes.byref(v)))
    return v.value


def wnnc_autotune(ctx, w: float = 0.002):
    """Time every tuned (tile shape, prefetch, split) setting on the current
    tree and keep the fastest.  Returns {(tpl, prefetch, split): ms}."""
    out = (TileTime * AUTOTUNE_CONFIGS)()
    _check(load_library().wnnc_autotune(ctx, float(w), out))
    return {(r.tpl, r.prefetch, r.split): r.ms for r in out}


def wnnc_build(ctx, P, c: float = 2.0, max_depth: int = 15, leaf_cap: int = 1) -> None:
    n = P.shape[0]
    opts = TreeOpts(float(c), int(max_depth), int(leaf_cap))
    _check(load_library().wnnc_build(ctx, _dev(P, "P", shape=(n, 3)), n, ctypes.byref(opts)))


def wnnc_winding(ctx, n, sigma, w: float, s_out) -> None:
    N = n.shape[0]
    _check(load_library().wnnc_winding(ctx, _dev(n, "n", shape=(N, 3)),
                                       _dev(sigma, "sigma", shape=(N,)), float(w),
                                       _dev(s_out, "s_out", shape=(N,))))


def wnnc_winding_at(ctx, n, sigma, w: float, Q, s_out) -> None:
    N = n.shape[0]
    M = Q.shape[0]
    _check(load_library().wnnc_winding_at(ctx, _dev(n, "n", shape=(N, 3)),
                                          _dev(sigma, "sigma", shape=(N,)), float(w),
                                          _dev(Q, "Q", shape=(M, 3)), M,
                                          _dev(s_out, "s_out", shape=(M,))))


def wnnc_gradient(ctx, n, sigma, w: float, grad_out) -> None:
    N = n.shape[0]
    _check(load_library().wnnc_gradient(ctx, _dev(n, "n", shape=(N, 3)),
                                        _dev(sigma, "sigma", shape=(N,)), float(w),
                                        _dev(grad_out, "grad_out", shape=(N, 3))))


def wnnc_adjoint(ctx, s, w: float, out) -> None:
    N = s.shape[0]
    _check(load_library().wnnc_adjoint(ctx, _dev(s, "s", shape=(N,)), float(w),
                                       _dev(out, "out", shape=(N, 3))))


def wnnc_energy(ctx, mu, w: float, gscale: float = 1.0, want_energy: bool = True,
                grad_out=None):
    """E = ||A_w mu - 1/2||^2 (returned when want_energy, else None) and, into
    grad_out (N,3) if given, gscale * dE/dmu = -2 gscale A_w^T (1/2 - A_w mu)."""
    N = mu.shape[0]
    e = ctypes.c_double(0.0)
    _check(load_library().wnnc_energy(ctx, _dev(mu, "mu", shape=(N, 3)), float(w), float(gscale),
                                      ctypes.byref(e) if want_energy else None,
                                      _dev(grad_out, "grad_out", shape=(N, 3))))
    return e.value if want_energy else None


def wnnc_orient(ctx, mu_out, mu0=None, iters: int = 40, w1: float = 0.002, w2: float = 0.016,
                start_iter: int = 1, stop_iter: int = 0, schedule: str = "linear",
                areas=None) -> None:
    N = mu_out.shape[0]
    ar = _dev(areas, "areas", shape=(N,))
    opts = OrientOpts(int(iters), float(w1), float(w2), int(start_iter), int(stop_iter),
                      SCHEDULES[schedule], ar.value if ar is not None else None)
    _check(load_library().wnnc_orient(ctx, ctypes.byref(opts), _dev(mu0, "mu0", shape=(N, 3)),
                                      _dev(mu_out, "mu_out", shape=(N, 3))))


def wnnc_normals(ctx, mu, scale: float, n_out, area_out=None) -> None:
    N = mu.shape[0]
    _check(load_library().wnnc_normals(ctx, _dev(mu, "mu", shape=(N, 3)), N, float(scale),
                                       _dev(n_out, "n_out", shape=(N, 3)),
                                       _dev(area_out, "area_out", shape=(N,))))


def wnnc_knn_features(ctx, feat_out, nbr_out=None) -> None:
    N = feat_out.shape[0]
    _check(load_library().wnnc_knn_features(ctx, _dev(feat_out, "feat_out", shape=(N, 48)),
                                            _dev(nbr_out, "nbr_out", dtype=torch.int32,
                                                 shape=(N, 16))))


def wnnc_winding_grad_x(ctx, mu, sigma, w: float, g, dx_out) -> None:
    """dL/dx of L = g . A_w(mu) with respect to the (normalized) points."""
    N = mu.shape[0]
    _check(load_library().wnnc_winding_grad_x(
        ctx, _dev(mu, "mu", shape=(N, 3)), _dev(sigma, "sigma", shape=(N,)), float(w),
        _dev(g, "g", shape=(N,)), _dev(dx_out, "dx_out", shape=(N, 3))))


def wnnc_winding_grad_x_noalloc(ctx, mu, sigma, w: float, g, dx_out) -> None:
    """wnnc_winding_grad_x with the library's static scratch: allocates no
    device memory (N <= NOALLOC_MAX_POINTS)."""
    N = mu.shape[0]
    _check(load_library().wnnc_winding_grad_x_noalloc(
        ctx, _dev(mu, "mu", shape=(N, 3)), _dev(sigma, "sigma", shape=(N,)), float(w),
        _dev(g, "g", shape=(N,)), _dev(dx_out, "dx_out", shape=(N, 3))))


def wnnc_gradient_grad_x(ctx, mu, sigma, w: float, v, dx_out) -> None:
    """dL/dx of L = v . grad F(mu) with respect to the (normalized) points."""
    N = mu.shape[0]
    _check(load_library().wnnc_gradient_grad_x(
        ctx, _dev(mu, "mu", shape=(N, 3)), _dev(sigma, "sigma", shape=(N,)), float(w),
        _dev(v, "v", shape=(N, 3)), _dev(dx_out, "dx_out", shape=(N, 3))))


def wnnc_set_far_field(ctx, order: int = 0, wsafe: bool = False) -> None:
    _check(load_library().wnnc_set_far_field(ctx, int(order), int(bool(wsafe))))


def wnnc_get_far_field(ctx) -> tuple:
    o, ws = ctypes.c_int(), ctypes.c_int()
    _check(load_library().wnnc_get_far_field(ctx, ctypes.byref(o), ctypes.byref(ws)))
    return o.value, bool(ws.value)


def wnnc_orient_preset(preset: str) -> dict:
    """iters, w1, w2 of one of the paper's parameter sets (PRESETS)."""
    o = OrientOpts()
    _check(load_library().wnnc_orient_preset(PRESETS[preset], ctypes.byref(o)))
    return {"iters": o.iters, "w1": o.w1, "w2": o.w2}


def wnnc_knn_areas(ctx, areas_out, k: int = 16) -> None:
    N = areas_out.shape[0]
    _check(load_library().wnnc_knn_areas(ctx, int(k), _dev(areas_out, "areas_out", shape=(N,))))


def wnnc_mlp_forward(ctx, params, feat, normals_out) -> None:
    N = feat.shape[0]
    _check(load_library().wnnc_mlp_forward(ctx, _dev(params, "params", shape=(MLP_PARAMS,)),
                                           _dev(feat, "feat", shape=(N, 48)), N,
                                           _dev(normals_out, "normals_out", shape=(N, 3))))


def wnnc_mlp_grad(ctx, params, feat, labels, grad_out, with_loss: bool = True):
    N = feat.shape[0]
    loss = ctypes.c_double(0.0)
    _check(load_library().wnnc_mlp_grad(ctx, _dev(params, "params", shape=(MLP_PARAMS,)),
                                        _dev(feat, "feat", shape=(N, 48)),
                                        _dev(labels, "labels", shape=(N, 3)), N,
                                        _dev(grad_out, "grad_out", shape=(MLP_PARAMS,)),
                                        ctypes.byref(loss) if with_loss else None))
    return loss.value if with_loss else None


def wnnc_mlp_adam(ctx, params, m, v, grad, step: int, lr: float = 1e-3, beta1: float = 0.9,
                  beta2: float = 0.999, eps: float = 1e-8) -> None:
    _check(load_library().wnnc_mlp_adam(ctx, _dev(params, "params", shape=(MLP_PARAMS,)),
                                        _dev(m, "m", shape=(MLP_PARAMS,)),
                                        _dev(v, "v", shape=(MLP_PARAMS,)),
                                        _dev(grad, "grad", shape=(MLP_PARAMS,)), int(step),
                                        float(lr), float(beta1), float(beta2), float(eps)))


def wnnc_warm_orient(ctx, params, mu_out, iters: int = 6, w1: float = 0.002, w2: float = 0.016,
                     max_disagree: float = 0.005, fallback_iters: int = 40,
                     fallback_w2: float = 0.016, max_pred_disagree: float = 0.4,
                     max_iters: int = 0, stop_frac: float = 0.0) -> dict:
    N = mu_out.shape[0]
    opts = WarmOpts(int(iters), float(w1), float(w2), float(max_disagree), int(fallback_iters),
                    float(fallback_w2), float(max_pred_disagree), int(max_iters), float(stop_frac))
    rep = WarmReport()
    _check(load_library().wnnc_warm_orient(ctx, _dev(params, "params", shape=(MLP_PARAMS,)),
                                           ctypes.byref(opts), _dev(mu_out, "mu_out", shape=(N, 3)),
                                           ctypes.byref(rep)))
    return dict(iterations=rep.iterations, fallback=bool(rep.fallback),
                max_disagree=rep.max_disagree, max_pred_disagree=rep.max_pred_disagree)


def wnnc_orient_energy(ctx, count: int, nclouds: int = 1):
    """Energies of the last orientation run: a list of `count` values for one
    cloud, or `count` lists of `nclouds` values."""
    buf = (ctypes.c_double * max(count * nclouds, 1))()
    _check(load_library().wnnc_orient_energy(ctx, buf, int(count)))
    if nclouds == 1:
        return [buf[i] for i in range(count)]
    return [[buf[i * nclouds + c] for c in range(nclouds)] for i in range(count)]


def wnnc_stats(ctx) -> dict:
    st = Stats()
    _check(load_library().wnnc_stats(ctx, ctypes.byref(st)))
    return st.as_dict()


def wnnc_reset_stats(ctx) -> None:
    _check(load_library().wnnc_reset_stats(ctx))


def wnnc_tree_export(ctx):
    """(depth, leaf, begin, end, perm) as numpy arrays (pre-order nodes)."""
    import numpy as np
    st = wnnc_stats(ctx)
    m, n = st["n_nodes"], st["n_points"]
    depth = np.zeros(m, np.int32)
    leaf = np.zeros(m, np.int32)
    begin = np.zeros(m, np.int64)
    end = np.zeros(m, np.int64)
    perm = np.zeros(n, np.int64)
    ptr = lambda a: ctypes.c_void_p(a.ctypes.data)
    _check(load_library().wnnc_tree_export(ctx, ptr(depth), ptr(leaf), ptr(begin), ptr(end),
                                           ptr(perm)))
    return depth, leaf, begin, end, perm


def wnnc_moments_export(ctx, nu):
    """(x_B, nu_B, W) per node for attribute nu ((N,3) or (N,) CUDA tensor)."""
    import numpy as np
    st = wnnc_stats(ctx)
    m = st["n_nodes"]
    dim = 3 if nu.dim() == 2 else 1
    xB = np.zeros((m, 3), np.float32)
    nuB = np.zeros((m, 3) if dim == 3 else (m,), np.float32)
    W = np.zeros(m, np.float32)
    ptr = lambda a: ctypes.c_void_p(a.ctypes.data)
    _check(load_library().wnnc_moments_export(ctx, _dev(nu, "nu"), dim, ptr(xB), ptr(nuB), ptr(W)))
    return xB, nuB, W


# ----------------------------------------------------------- wrapper --

@dataclass
class Normalization:
    center: tuple
    scale: float


class Context:
    """One library context bound to a device and (by default) torch's current
    stream at creation time."""

    def __init__(self, device: int = 0, stream=None):
        self.device = int(device)
        self._h = wnnc_create(self.device, stream)
        self.n = 0

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            wnnc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_flags(self, flags: int) -> None:
        wnnc_set_flags(self._h, flags)

    def set_stream(self, stream=None) -> None:
        wnnc_set_stream(self._h, stream)

    def normalize(self, P):
        out = torch.empty_like(P)
        c, s = wnnc_normalize(self._h, P, out)
        return out, Normalization(c, s)

    def build(self, P_norm, c: float = 2.0, max_depth: int = 15, leaf_cap: int = 1) -> None:
        wnnc_build(self._h, P_norm, c, max_depth, leaf_cap)
        self.n = int(P_norm.shape[0])
        self.nclouds = 1

    def normalize_batched(self, P, offsets):
        out = torch.empty_like(P)
        cs = wnnc_normalize_batched(self._h, P, out, offsets)
        return out, [Normalization(c, s) for c, s in cs]

    def build_batched(self, P_norm, offsets, c: float = 2.0, max_depth: int = 15,
                      leaf_cap: int = 1) -> None:
        wnnc_build_batched(self._h, P_norm, offsets, c, max_depth, leaf_cap)
        self.n = int(P_norm.shape[0])
        self.nclouds = len(offsets) - 1

    def set_tile(self, tpl: int) -> None:
        wnnc_set_tile(self._h, tpl)

    def set_defer(self, lanes: int) -> None:
        _check(load_library().wnnc_set_defer(self._h, int(lanes)))

    def defer(self) -> int:
        v = ctypes.c_int(0)
        _check(load_library().wnnc_get_defer(self._h, ctypes.byref(v)))
        return v.value

    def set_prefetch(self, on: bool) -> None:
        wnnc_set_prefetch(self._h, on)

    def tile(self) -> int:
        return wnnc_get_tile(self._h)

    def prefetch(self) -> bool:
        return bool((wnnc_stats(self._h)["tile"] >> 8) & 1)

    def set_split(self, visits: int) -> None:
        wnnc_set_split(self._h, visits)

    def split(self) -> int:
        return wnnc_get_split(self._h)

    def autotune(self, w: float = 0.002):
        return wnnc_autotune(self._h, w)

    def winding(self, mu, w: float, sigma=None):
        out = torch.empty(mu.shape[0], device=mu.device, dtype=torch.float32)
        wnnc_winding(self._h, mu, sigma, w, out)
        return out

    def winding_at(self, mu, w: float, Q, sigma=None):
        """F(Q_k; mu) at query points Q (M,3) in the normalized frame."""
        out = torch.empty(Q.shape[0], device=Q.device, dtype=torch.float32)
        wnnc_winding_at(self._h, mu, sigma, w, Q, out)
        return out

    def gradient(self, mu, w: float, sigma=None):
        out = torch.empty_like(mu)
        wnnc_gradient(self._h, mu, sigma, w, out)
        return out

    def adjoint(self, s, w: float):
        out = torch.empty(s.shape[0], 3, device=s.device, dtype=torch.float32)
        wnnc_adjoint(self._h, s, w, out)
        return out

    def orient(self, iters: int = 40, w1: float = 0.002, w2: float = 0.016, mu0=None,
               start_iter: int = 1, stop_iter: int = 0, out=None, schedule: str = "linear",
               areas=None, preset: str | None = None):
        """Alg. 3; `preset` (a PRESETS name) replaces iters, w1 and w2."""
        if preset is not None:
            p = wnnc_orient_preset(preset)
            iters, w1, w2 = p["iters"], p["w1"], p["w2"]
        if out is None:
            out = torch.empty(self.n, 3, device=f"cuda:{self.device}", dtype=torch.float32)
        wnnc_orient(self._h, out, mu0, iters, w1, w2, start_iter, stop_iter, schedule, areas)
        return out

    def normals(self, mu, scale: float = 1.0, with_area: bool = False):
        nrm = torch.empty_like(mu)
        area = torch.empty(mu.shape[0], device=mu.device, dtype=torch.float32) if with_area else None
        wnnc_normals(self._h, mu, scale, nrm, area)
        return (nrm, area) if with_area else nrm

    def warm_orient(self, params, out=None, **kw):
        if out is None:
            out = torch.empty(self.n, 3, device=f"cuda:{self.device}", dtype=torch.float32)
        rep = wnnc_warm_orient(self._h, params, out, **kw)
        return out, rep

    def features(self, with_neighbours: bool = False):
        feat = torch.empty(self.n, 48, device=f"cuda:{self.device}", dtype=torch.float32)
        nbr = (torch.empty(self.n, 16, device=f"cuda:{self.device}", dtype=torch.int32)
               if with_neighbours else None)
        wnnc_knn_features(self._h, feat, nbr)
        return (feat, nbr) if with_neighbours else feat

    def winding_grad_x(self, mu, w: float, g, sigma=None):
        """Gradient of g . A_w(mu) with respect to the normalized points."""
        out = torch.empty(mu.shape[0], 3, device=mu.device, dtype=torch.float32)
        wnnc_winding_grad_x(self._h, mu, sigma, w, g, out)
        return out

    def gradient_grad_x(self, mu, w: float, v, sigma=None):
        """Gradient of v . grad F(mu) with respect to the normalized points."""
        out = torch.empty(mu.shape[0], 3, device=mu.device, dtype=torch.float32)
        wnnc_gradient_grad_x(self._h, mu, sigma, w, v, out)
        return out

    def set_far_field(self, order: int = 0, wsafe: bool = False) -> None:
        """Far-field order (0 = Alg. 4, 1, 2) and the cutoff-safe acceptance."""
        wnnc_set_far_field(self._h, order, wsafe)

    def far_field(self) -> tuple:
        return wnnc_get_far_field(self._h)

    def knn_areas(self, k: int = 16, out=None):
        """kNN local areas of every point (normalized frame, caller order)."""
        if out is None:
            out = torch.empty(self.n, device=f"cuda:{self.device}", dtype=torch.float32)
        _dev(out, "out", shape=(self.n,))
        wnnc_knn_areas(self._h, out, k)
        return out

    def energy(self, count: int):
        return wnnc_orient_energy(self._h, count, getattr(self, "nclouds", 1))

    def stats(self) -> dict:
        return wnnc_stats(self._h)

    def reset_stats(self) -> None:
        wnnc_reset_stats(self._h)

    def tree(self):
        return wnnc_tree_export(self._h)

    def moments(self, nu):
        return wnnc_moments_export(self._h, nu)


def orient_points(P, iters: int = 40, w1: float = 0.002, w2: float = 0.016, c: float = 2.0,
                  max_depth: int = 15, device: int = 0):
    """Normalize, build and run the WNNC iteration on a (N,3) CUDA tensor.
    Returns (mu in the normalized frame, unit normals, Normalization)."""
    ctx = Context(device)
    try:
        x, norm = ctx.normalize(P.contiguous().float())
        ctx.build(x, c, max_depth)
        mu = ctx.orient(iters, w1, w2)
        nrm = ctx.normals(mu)
        return mu, nrm, norm
    finally:
        ctx.close()
