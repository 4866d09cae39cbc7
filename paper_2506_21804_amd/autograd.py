"""torch.autograd wrapper of the porosity-gradient problem.

``LbmObjective.apply(phi, case, storage, T, planes, nsnap)`` runs T steps of
the homogenized LB update from the case's initial state with porosity phi
(Sec. 2.2, Eq. (12)) and returns the terminal objective
J = c_s^2 (<rho>_{x=p0} - <rho>_{x=p1}) + <rho |u|^2 / 2>, or with
``mean=True`` its average over the states of steps 1..T.  When phi requires
a gradient, the forward pass already runs the library's checkpointed reverse
sweep (``lbm_gradient``: binomial schedule over ``nsnap`` snapshot slots,
hand-written adjoint kernel) and keeps dJ/dphi for the backward pass.  All
arithmetic runs in the HIP library.
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from . import Lattice, lbm_gradient, lbm_gradient_mean, lbm_state_bytes


class LbmObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, case, storage="f32", T=400, planes=None, nsnap=20, mean=False):
        if planes is None:
            planes = case.extra["planes"]
        c = copy.copy(case)
        c.porosity = phi.detach().to("cpu", torch.float64).numpy().reshape(-1).copy()
        lat = Lattice(c, storage=storage)
        if phi.requires_grad:
            lam = lat.new_adjoint()
            grad = lat.new_gradient()
            snaps = torch.empty(nsnap * lbm_state_bytes(lat.ctx), dtype=torch.uint8, device="cuda")
            J, _ = (lbm_gradient_mean if mean else lbm_gradient)(lat.ctx, T, planes, snaps, nsnap, lam, grad)
            ctx.save_for_backward(grad.to(phi.device, phi.dtype).reshape(phi.shape))
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
        (grad,) = ctx.saved_tensors
        return gJ.to(grad.dtype) * grad, None, None, None, None, None, None


def objective(phi, case, storage="f32", T=400, planes=None, nsnap=20, mean=False):
    return LbmObjective.apply(phi, case, storage, T, planes, nsnap, mean)
