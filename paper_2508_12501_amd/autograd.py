"""Reverse-mode differentiation through the multigrid solve and the porous-convection rollout
of arXiv 2508.12501 (the solve of Sec. 3.1 and the model of Sec. 3.2; the paper does not
differentiate them, so this is an extension: the loss gradient with respect to the permeability
field flows back through the DEC operators and the linear solves).

Both wrappers are ``torch.autograd.Function``s whose forward and backward passes are calls of
the library's entry points (``mg_pcg`` / ``mg_pcg_adjoint``, ``porous_step`` /
``porous_step_adjoint``, and ``mg_hierarchy_set_log_coeff`` / ``mg_hierarchy_coeff_grad_log``
for k = exp(g) and its chain rule); nothing here does arithmetic on the fields beyond
zero-filling the gradient buffers.

The hierarchy holds one vertex coefficient at a time.  Each forward and each backward pass
sets the coefficient it was called with, so interleaving several graphs on one hierarchy is
correct (at the cost of one coefficient upload per pass).
"""
from __future__ import annotations

import torch

from . import (mg_hierarchy_coeff_grad_log, mg_hierarchy_set_log_coeff,
               mg_hierarchy_set_vertex_coeff, mg_opts_default, mg_pcg, mg_pcg_adjoint,
               porous_params_make, porous_step, porous_step_adjoint)


def _f64(t, name):
    if t.dtype != torch.float64 or not t.is_cuda:
        raise ValueError(f"{name} must be a float64 tensor on the GPU")
    return t.detach().contiguous()


class MGSolve(torch.autograd.Function):
    """u = A(k)^{-1} b by MG-PCG; gradients dJ/db = A^{-1} dJ/du and dJ/dk at the vertices.
    k = None keeps the unit coefficient (no gradient for it)."""

    @staticmethod
    def forward(ctx, hier, opts, b, k):
        b = _f64(b, "b")
        if k is not None:
            k = _f64(k, "k")
        mg_hierarchy_set_vertex_coeff(hier.h, k)
        u = torch.zeros_like(b)
        mg_pcg(hier.h, opts, b, u)
        ctx.hier, ctx.opts = hier, opts
        ctx.save_for_backward(u, k if k is not None else torch.empty(0))
        ctx.has_k = k is not None
        return u

    @staticmethod
    def backward(ctx, grad_u):
        u, k = ctx.saved_tensors
        k = k if ctx.has_k else None
        mg_hierarchy_set_vertex_coeff(ctx.hier.h, k)
        gb = torch.zeros_like(u)
        want_k = ctx.has_k and ctx.needs_input_grad[3]
        gk = torch.zeros_like(u) if want_k else None
        mg_pcg_adjoint(ctx.hier.h, ctx.opts, u, grad_u.contiguous(), gb, gk)
        return None, None, gb if ctx.needs_input_grad[2] else None, gk


def mg_solve_diff(hier, b, k=None, opts=None):
    """Differentiable solve of A(k) u = b (see MGSolve)."""
    return MGSolve.apply(hier, opts if opts is not None else mg_opts_default(rtol=1e-12), b, k)


class PorousRollout(torch.autograd.Function):
    """T_N after `steps` forward-Euler steps of the porous model from T_0 with permeability
    k = exp(g).  The forward pass keeps T every `ckpt` steps; the backward pass recomputes each
    segment from its checkpoint (keeping the segment's temperatures and pressures) and runs the
    step adjoints in reverse.  Returns gradients for T_0 and g."""

    @staticmethod
    def forward(ctx, hier, prm, T0, g, steps, ckpt):
        T0 = _f64(T0, "T0")
        g = _f64(g, "g")
        mg_hierarchy_set_log_coeff(hier.h, g)
        ckpt = int(ckpt) if ckpt else int(steps)
        saved = {0: T0.clone()}
        T, Tn = T0.clone(), torch.empty_like(T0)
        for n in range(steps):
            porous_step(hier.h, prm, T, Tn)
            T, Tn = Tn, T
            if (n + 1) % ckpt == 0 and n + 1 < steps:
                saved[n + 1] = T.clone()
        ctx.hier, ctx.prm, ctx.steps, ctx.ckpt, ctx.saved = hier, prm, int(steps), ckpt, saved
        ctx.save_for_backward(g)
        return T

    @staticmethod
    def backward(ctx, grad_T):
        (g,) = ctx.saved_tensors
        hier, prm = ctx.hier, ctx.prm
        mg_hierarchy_set_log_coeff(hier.h, g)
        lam = grad_T.detach().contiguous().clone()
        lam_n = torch.empty_like(lam)
        gk = torch.zeros_like(lam)
        for s0 in sorted(ctx.saved, reverse=True):
            s1 = min(s0 + ctx.ckpt, ctx.steps)
            Ts, Ps = [ctx.saved[s0]], []
            for _ in range(s0, s1):
                p = torch.empty_like(lam)
                nxt = torch.empty_like(lam)
                porous_step(hier.h, prm, Ts[-1], nxt, p)
                Ps.append(p)
                Ts.append(nxt)
            for i in range(s1 - s0 - 1, -1, -1):
                porous_step_adjoint(hier.h, prm, Ts[i], Ps[i], lam, lam_n, gk)
                lam, lam_n = lam_n, lam
        ctx.saved = None
        gT0 = lam if ctx.needs_input_grad[2] else None
        gg = None
        if ctx.needs_input_grad[3]:
            gg = torch.zeros_like(gk)
            mg_hierarchy_coeff_grad_log(hier.h, gk, gg)
        return None, None, gT0, gg, None, None


def porous_rollout(hier, T0, g, steps, Ra, phi, dt, ckpt=20, solve=None):
    """Differentiable rollout (see PorousRollout)."""
    prm = porous_params_make(Ra, phi, dt, solve if solve is not None else mg_opts_default(rtol=1e-12))
    return PorousRollout.apply(hier, prm, T0, g, int(steps), int(ckpt))
