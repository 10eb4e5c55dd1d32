"""Differentiable winding numbers: autograd Functions over the C ABI.

The adjoint operator is the backward of the winding-number operator
(Sec. 4.5, last paragraph: A^T is exactly the backward function of A):

* ``winding(ctx, mu, w)``   s = A_w(mu)          backward: g -> A_w^T g
* ``adjoint(ctx, s, w)``    v = A_w^T s          backward: g -> A_w g
* ``gradient(ctx, mu, w)``  grad F = -G_w(mu)    backward: g -> -G_w g
  (G is symmetric: HPhi is an even, symmetric matrix field)
* ``pgr_energy(ctx, mu, w)``  E = ||A_w mu - 1/2||^2   backward: g -> -2 g r
  (r of Alg. 2; both from wnnc_energy)
* ``winding_at_points(ctx, x, mu, w)``  s = A_w(mu) on the tree built from
  the normalized points x; differentiable in x and mu (an extension:
  backward in x is wnnc_winding_grad_x, g -> g grad F + p)
* ``gradient_at_points(ctx, x, mu, w)``  grad F = -G_w(mu) likewise (backward
  in x is wnnc_gradient_grad_x)

All three evaluate with the context's treecode; every forward and backward
runs in the library's kernels (argument marshalling only here).  With the
treecode the backward is the treecode of the transposed operator, as in the
paper; it equals the exact gradient of the treecode forward only up to the
treecode's approximation error, because the representatives depend on |nu|.
"""
from __future__ import annotations

import torch

from . import (wnnc_adjoint, wnnc_build, wnnc_energy, wnnc_gradient, wnnc_gradient_grad_x,
               wnnc_winding, wnnc_winding_grad_x)


def _prep(t):
    return t.detach().contiguous().float()


class WindingNumber(torch.autograd.Function):
    @staticmethod
    def forward(fctx, handle, mu, w):
        fctx.handle, fctx.w = handle, float(w)
        out = torch.empty(mu.shape[0], device=mu.device, dtype=torch.float32)
        wnnc_winding(handle, _prep(mu), None, fctx.w, out)
        return out

    @staticmethod
    def backward(fctx, g):
        gm = torch.empty(g.shape[0], 3, device=g.device, dtype=torch.float32)
        wnnc_adjoint(fctx.handle, _prep(g), fctx.w, gm)
        return None, gm, None


class WindingAdjoint(torch.autograd.Function):
    @staticmethod
    def forward(fctx, handle, s, w):
        fctx.handle, fctx.w = handle, float(w)
        out = torch.empty(s.shape[0], 3, device=s.device, dtype=torch.float32)
        wnnc_adjoint(handle, _prep(s), fctx.w, out)
        return out

    @staticmethod
    def backward(fctx, g):
        gs = torch.empty(g.shape[0], device=g.device, dtype=torch.float32)
        wnnc_winding(fctx.handle, _prep(g), None, fctx.w, gs)
        return None, gs, None


class WindingGradient(torch.autograd.Function):
    @staticmethod
    def forward(fctx, handle, mu, w):
        fctx.handle, fctx.w = handle, float(w)
        out = torch.empty_like(mu, dtype=torch.float32)
        wnnc_gradient(handle, _prep(mu), None, fctx.w, out)
        return out

    @staticmethod
    def backward(fctx, g):
        gm = torch.empty_like(g, dtype=torch.float32)
        wnnc_gradient(fctx.handle, _prep(g), None, fctx.w, gm)
        return None, gm, None


def _handle(ctx):
    return ctx.handle if hasattr(ctx, "handle") else ctx


def winding(ctx, mu, w: float):
    """s = A_w(mu) at the points of ctx's tree; differentiable in mu."""
    return WindingNumber.apply(_handle(ctx), mu, w)


def adjoint(ctx, s, w: float):
    """A_w^T s; differentiable in s."""
    return WindingAdjoint.apply(_handle(ctx), s, w)


def gradient(ctx, mu, w: float):
    """grad F(x_i; mu) = -G_w(mu)_i; differentiable in mu."""
    return WindingGradient.apply(_handle(ctx), mu, w)


class PgrEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, handle, mu, w):
        fctx.handle, fctx.w = handle, float(w)
        m = _prep(mu)
        fctx.save_for_backward(m)
        E = wnnc_energy(handle, m, fctx.w)
        return torch.tensor(E, dtype=torch.float64, device=mu.device)

    @staticmethod
    def backward(fctx, g):
        (m,) = fctx.saved_tensors
        gm = torch.empty_like(m)
        # the chain-rule factor goes to the library as a host scalar
        wnnc_energy(fctx.handle, m, fctx.w, gscale=float(g), want_energy=False, grad_out=gm)
        return None, gm, None


def pgr_energy(ctx, mu, w: float):
    """E(mu) = ||A_w mu - b||^2 with b = 1/2 (the energy of Alg. 2's gradient
    step), evaluated by the library (wnnc_energy); its gradient is
    2 A_w^T (A_w mu - b) = -2 r of Alg. 2, also from the library."""
    return PgrEnergy.apply(_handle(ctx), mu, w)


class WindingPositions(torch.autograd.Function):
    @staticmethod
    def forward(fctx, handle, x, mu, w, c, max_depth):
        fctx.handle, fctx.w = handle, float(w)
        wnnc_build(handle, _prep(x), float(c), int(max_depth))
        m = _prep(mu)
        out = torch.empty(m.shape[0], device=m.device, dtype=torch.float32)
        wnnc_winding(handle, m, None, fctx.w, out)
        fctx.save_for_backward(m)
        return out

    @staticmethod
    def backward(fctx, g):
        (m,) = fctx.saved_tensors
        gg = _prep(g)
        gx = torch.empty(m.shape[0], 3, device=g.device, dtype=torch.float32)
        wnnc_winding_grad_x(fctx.handle, m, None, fctx.w, gg, gx)
        gm = torch.empty(m.shape[0], 3, device=g.device, dtype=torch.float32)
        wnnc_adjoint(fctx.handle, gg, fctx.w, gm)
        return None, gx, gm, None, None, None


def winding_at_points(ctx, x, mu, w: float, c: float = 2.0, max_depth: int = 15):
    """s = A_w(mu) at the normalized points x, building ctx's tree on x;
    differentiable in x and in mu.  The backward reuses the tree of the
    forward, so call backward before the next build on ctx."""
    return WindingPositions.apply(_handle(ctx), x, mu, w, c, max_depth)


class GradientPositions(torch.autograd.Function):
    @staticmethod
    def forward(fctx, handle, x, mu, w, c, max_depth):
        fctx.handle, fctx.w = handle, float(w)
        wnnc_build(handle, _prep(x), float(c), int(max_depth))
        m = _prep(mu)
        out = torch.empty_like(m)
        wnnc_gradient(handle, m, None, fctx.w, out)
        fctx.save_for_backward(m)
        return out

    @staticmethod
    def backward(fctx, g):
        (m,) = fctx.saved_tensors
        gg = _prep(g)
        gx = torch.empty_like(m)
        wnnc_gradient_grad_x(fctx.handle, m, None, fctx.w, gg, gx)
        gm = torch.empty_like(m)
        wnnc_gradient(fctx.handle, gg, None, fctx.w, gm)
        return None, gx, gm, None, None, None


def gradient_at_points(ctx, x, mu, w: float, c: float = 2.0, max_depth: int = 15):
    """grad F = -G_w(mu) at the normalized points x, building ctx's tree on
    x; differentiable in x and in mu (as winding_at_points)."""
    return GradientPositions.apply(_handle(ctx), x, mu, w, c, max_depth)

