"""torch.autograd.Function for receiver pressures as a function of the
per-cell sound speed and density (argument marshalling only: every step runs
in libvsie.so).

Forward: set the materials, solve A P = b for the plane-wave incidences,
evaluate p_rec = p_inc - E P at the receivers (the representation formula,
section 2.3.1 of the paper).  Backward (for a real loss, given its
conjugate-Wirtinger gradient rho with respect to p_rec, PyTorch's complex
convention): adjoint right-hand side E^H rho, adjoint solve A^H lam = E^H rho,
source-side sums, and the chain rule to (c, rho) -- vsie_param_gradient.
"""
from __future__ import annotations

import numpy as np
import torch

from . import VSIE_FP64, Problem


class ReceiverPressure(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, rho, problem: Problem, n_vol: int, dirs, receivers, f: int, prec: int,
                tol: float, block: bool):
        rho_f, c_f = rho.detach().contiguous(), c.detach().contiguous()
        problem.set_materials(rho_f, c_f)
        b = problem.plane_wave(np.atleast_2d(dirs), f=f)
        P, info = problem.solve(b, f=f, prec=prec, tol=tol, block=block)
        p_rec = problem.plane_wave_at(receivers, dirs, f=f) - problem.field(receivers, P, f=f)
        ctx.problem, ctx.n_vol, ctx.receivers, ctx.f, ctx.prec, ctx.tol, ctx.block = (
            problem, n_vol, receivers, f, prec, tol, block)
        ctx.info = info
        # the adjoint operator and the chain rule read the problem's current
        # materials: remember which ones this forward used
        ctx.version = problem.material_version
        ctx.save_for_backward(P, rho_f.clone(), c_f.clone())
        return p_rec

    @staticmethod
    def backward(ctx, grad_out):
        P, rho_f, c_f = ctx.saved_tensors
        pb: Problem = ctx.problem
        if pb.material_version != ctx.version:
            # another forward (or set_materials) changed the problem since:
            # restore this forward's materials
            pb.set_materials(rho_f, c_f)
            ctx.version = pb.material_version
        resid = grad_out.contiguous()
        zR, ZR = pb.source_sums(resid, f=ctx.f, targets=ctx.receivers)
        rhs = pb.adjoint_rhs(zR, ZR, f=ctx.f)
        lam, ctx.adj_info = pb.solve(rhs, f=ctx.f, prec=ctx.prec, adjoint=True, tol=ctx.tol, block=ctx.block)
        z, Z = pb.source_sums(lam, f=ctx.f)
        gc, grho = pb.param_gradient(P, lam, z, Z, zR, ZR, ctx.n_vol, f=ctx.f)
        return gc, grho, None, None, None, None, None, None, None, None


def receiver_pressure(problem: Problem, n_vol: int, c, rho, dirs, receivers, f=0, prec=VSIE_FP64,
                      tol=1e-12, block=False):
    """Receiver pressures (Q, n_rec) for Q plane waves; differentiable in c, rho.
    block selects block GMRES for the forward and adjoint solves."""
    return ReceiverPressure.apply(c, rho, problem, n_vol, np.atleast_2d(dirs), receivers, f, prec, tol,
                                  block)
