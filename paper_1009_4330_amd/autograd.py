"""Forces as differentiable torch functions: LJForces (eps, sigma) and
SCForces (Sutton-Chen eps, a, c).

forward evaluates F(x; params) with md_compute_forces over a fixed neighbour
list; backward(u) calls the hand-written adjoint md_force_vjp, which returns
(dF/dx)^T u = -H u and the parameter gradients.  The pair set is the listed
pairs inside rc (rc does not scale with sigma or a), frozen at the list the
function was given.
"""
from __future__ import annotations

import torch

from . import md


class LJForces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, eps, sigma, box, nl, rc, prec, ws):
        pot = md.lj_potential(rc, float(eps), float(sigma), 0)
        f = torch.empty_like(x)
        md.md_compute_forces(pot, x, box, nl, prec, md.MD_KERNEL_AUTO, 0, f, None, ws)
        ctx.save_for_backward(x)
        ctx.meta = (box, nl, rc, prec, ws, float(eps), float(sigma))
        return f

    @staticmethod
    def backward(ctx, u):
        (x,) = ctx.saved_tensors
        box, nl, rc, prec, ws, eps, sigma = ctx.meta
        pot = md.lj_potential(rc, eps, sigma, 0)
        gx = torch.empty_like(x)
        gp = torch.empty(2, dtype=torch.float64, device=x.device)
        md.md_force_vjp(pot, x, box, nl, prec, u.contiguous(), gx, gp, ws)
        return gx, gp[0], gp[1], None, None, None, None, None


def lj_forces(x, eps, sigma, box, nl, rc, prec=md.MD_FP64, ws=None):
    """F(x; eps, sigma) [3][n]; eps and sigma are 0-d tensors (may require grad)."""
    if ws is None:
        ws = md.workspace(x.shape[1], box, max(rc, nl.c.rl))
    return LJForces.apply(x, eps, sigma, box, nl, rc, prec, ws)


class SCForces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, eps, a, c, box, nl, rc, nexp, mexp, prec, ws):
        pot = md.sc_potential(rc, float(eps), float(a), float(c), nexp, mexp)
        f = torch.empty_like(x)
        md.md_compute_forces(pot, x, box, nl, prec, md.MD_KERNEL_AUTO, 0, f, None, ws)
        ctx.save_for_backward(x)
        ctx.meta = (box, nl, rc, nexp, mexp, prec, ws, float(eps), float(a), float(c))
        return f

    @staticmethod
    def backward(ctx, u):
        (x,) = ctx.saved_tensors
        box, nl, rc, nexp, mexp, prec, ws, eps, a, c = ctx.meta
        pot = md.sc_potential(rc, eps, a, c, nexp, mexp)
        gx = torch.empty_like(x)
        gp = torch.empty(3, dtype=torch.float64, device=x.device)
        md.md_force_vjp(pot, x, box, nl, prec, u.contiguous(), gx, gp, ws)
        return gx, gp[0], gp[1], gp[2], None, None, None, None, None, None, None


def sc_forces(x, eps, a, c, box, nl, rc, nexp, mexp, prec=md.MD_FP64, ws=None):
    """Sutton-Chen F(x; eps, a, c) [3][n]; eps, a, c are 0-d tensors (may
    require grad); nexp, mexp the integer exponents."""
    if ws is None:
        ws = md.workspace(x.shape[1], box, max(rc, nl.c.rl))
    return SCForces.apply(x, eps, a, c, box, nl, rc, nexp, mexp, prec, ws)
