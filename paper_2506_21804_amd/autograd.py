"""torch.autograd wrapper of the porosity-gradient problem.

``objective(phi, case, storage, T, planes, nsnap, mean, cs)`` runs T steps of
the homogenized LB update from the case's initial state with porosity phi
(Sec. 2.2, Eq. (12)) and, when ``cs`` is given, the per-cell Smagorinsky
constant cs (Sec. 2.3), and returns the terminal objective
J = c_s^2 (<rho>_{x=p0} - <rho>_{x=p1}) + <rho |u|^2 / 2>, or with
``mean=True`` its average over the states of steps 1..T.  When phi or cs
requires a gradient, the forward pass already runs the library's
checkpointed reverse sweep (``lbm_gradient`` / ``lbm_gradient_cs``: binomial
schedule over ``nsnap`` snapshot slots, hand-written adjoint kernels) and
keeps dJ/dphi and dJ/dC_S for the backward pass.  All arithmetic runs in the
HIP library.
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from . import Lattice, lbm_gradient, lbm_gradient_cs, lbm_gradient_mean, lbm_state_bytes


class LbmObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, cs, case, storage="f32", T=400, planes=None, nsnap=20, mean=False):
        if planes is None:
            planes = case.extra["planes"]
        c = copy.copy(case)
        c.porosity = phi.detach().to("cpu", torch.float64).numpy().reshape(-1).copy()
        lat = Lattice(c, storage=storage, cs_field=cs is not None)
        if cs is not None:
            lat.set_smagorinsky(cs.detach().to("cuda", torch.float64).reshape(-1).contiguous())
        want_cs = cs is not None and cs.requires_grad
        ctx.has_cs = cs is not None
        if phi.requires_grad or want_cs:
            lam = lat.new_adjoint()
            grad = lat.new_gradient()
            snaps = torch.empty(nsnap * lbm_state_bytes(lat.ctx), dtype=torch.uint8, device="cuda")
            if want_cs:
                gcs = lat.new_gradient()
                J, _ = lbm_gradient_cs(lat.ctx, T, planes, snaps, nsnap, lam, grad, gcs, mean=mean)
                gcs = gcs.to(cs.device, cs.dtype).reshape(cs.shape)
            else:
                J, _ = (lbm_gradient_mean if mean else lbm_gradient)(lat.ctx, T, planes, snaps, nsnap, lam, grad)
                gcs = torch.zeros(0)
            ctx.save_for_backward(grad.to(phi.device, phi.dtype).reshape(phi.shape), gcs)
        elif mean:
            J = 0.0
            for _ in range(T):
                lat.step(1)
                J += lat.objective(planes)
            J /= T
        else:
            lat.step(T)
            J = lat.objective(planes)
        return torch.tensor(J, dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(ctx, gJ):
        grad, gcs = ctx.saved_tensors
        g_cs = gJ.to(gcs.dtype) * gcs if (ctx.has_cs and gcs.numel()) else None
        return gJ.to(grad.dtype) * grad, g_cs, None, None, None, None, None, None


def objective(phi, case, storage="f32", T=400, planes=None, nsnap=20, mean=False, cs=None):
    return LbmObjective.apply(phi, cs, case, storage, T, planes, nsnap, mean)
