"""Differentiable Wilson-Dirac solve x = D[U]^{-1} b as a torch.autograd.Function.

Forward: x = D^{-1} b through the library's solver (default: BiCGStab with an
FP32 inner solve inside FP64 refinement); x is kept in the autograd context
(the solution checkpoint) unless ``checkpoint=False``, in which case the
backward re-solves for it.

Backward, for upstream g = dL/dRe x + i dL/dIm x (PyTorch's convention for a
real loss):
  * adjoint   mu = D^{-dag} g, solved by the library on D^dag = gamma5 D gamma5;
  * grad_b    = mu  (since dL = Re<g, D^{-1} db> = Re<D^{-dag} g, db>);
  * grad_U    from the library's force kernel: dL = Re sum Tr[dU G] with
    G_mu(x) = kappa s_mu(x) [ sum_spin ((1-g_mu) x(x+mu)) mu(x)^dag
                            + sum_spin mu(x+mu) ((1+g_mu) x(x))^dag ]
    (differentiating D = 1 - kappa H link by link).  ``link_grad="su3"``
    returns the tangent gradient i P U with P = TH(i U G), whose component
    along U -> exp(i w T) U is Tr[T P]; ``link_grad="complex"`` returns the
    unconstrained complex gradient G^dag.
Every step (solves, packing, force, projection) runs in the HIP library; torch
provides memory and the stream.
"""
from __future__ import annotations

import torch

from . import wilson as W


class WilsonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, b, kappa, method="bicgstab", precision="mixed-f32", tol=1e-10, bc=(1, 1, 1, -1),
                link_grad="su3", checkpoint=True):
        if b.dim() != 6:
            raise ValueError("WilsonSolve takes one right-hand side (Lt, Lz, Ly, Lx, 4, 3)")
        hi = W.Operator.create(U.detach(), kappa, W.WL_F64, bc)
        lo = None
        if precision.startswith("mixed-"):
            lo = W.Operator.create(U.detach(), kappa, W.PREC[precision.split("-", 1)[1]], bc)
        elif precision != "f64":
            raise ValueError("precision must be f64 or mixed-*")
        x, st = W.solve(None, b.detach(), kappa, method=method, precision=precision, tol=tol, bc=bc,
                        ops=(hi, lo), return_stats=True)
        if not st["converged"]:
            raise RuntimeError(f"forward solve did not converge: {st}")
        ctx.ops = (hi, lo)
        ctx.cfg = (kappa, method, precision, tol, bc, link_grad, checkpoint)
        ctx.b = None if checkpoint else b.detach()
        ctx.save_for_backward(x if checkpoint else torch.empty(0))
        return x

    @staticmethod
    def backward(ctx, g):
        kappa, method, precision, tol, bc, link_grad, checkpoint = ctx.cfg
        hi, lo = ctx.ops
        (x,) = ctx.saved_tensors
        if not checkpoint:
            x = W.solve(None, ctx.b, kappa, method=method, precision=precision, tol=tol, bc=bc, ops=(hi, lo))
        g = g.contiguous()
        mu, st = W.solve(None, g, kappa, method=method, precision=precision, tol=tol, bc=bc, ops=(hi, lo),
                         dagger=True, return_stats=True)
        if not st["converged"]:
            raise RuntimeError(f"adjoint solve did not converge: {st}")
        grad_U = None
        if ctx.needs_input_grad[0]:
            xp = hi.pack(x)
            mp = hi.pack(mu)
            grad_U = W.gauge_force(hi, xp, mp, project=2 if link_grad == "su3" else 0)
        grad_b = mu if ctx.needs_input_grad[1] else None
        return grad_U, grad_b, None, None, None, None, None, None, None


def wilson_solve(U, b, kappa, method="bicgstab", precision="mixed-f32", tol=1e-10, bc=(1, 1, 1, -1),
                 link_grad="su3", checkpoint=True):
    """Differentiable x = D[U]^{-1} b (see WilsonSolve)."""
    return WilsonSolve.apply(U, b, kappa, method, precision, tol, tuple(bc), link_grad, checkpoint)

