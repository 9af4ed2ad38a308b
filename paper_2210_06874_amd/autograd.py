"""The pseudofermion action as a differentiable function of the Hubbard field.

S[phi] = chi^dag (M M^dag)^{-1} chi   (Sec. 2, eq. "hamiltonian")

forward:  x = CG(phi, chi) on the device, S = Re chi^dag x.
backward: dS/dphi from the adjoint force kernel, which reuses the CG solution x
          and recomputes E x per slice; nothing is stored per slice.
"""
from __future__ import annotations

import torch


class PseudofermionAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, chi, hub, tol=1e-10, prec="fp64", max_iter=100000, reliable_every=50):
        res = hub.cg_solve(phi, chi, tol=tol, max_iter=max_iter, prec=prec, reliable_every=reliable_every)
        S = hub.action(chi, res.x)
        ctx.hub = hub
        ctx.save_for_backward(phi, res.x)
        ctx.cg = res
        return S

    @staticmethod
    def backward(ctx, grad_S):
        phi, x = ctx.saved_tensors
        g = ctx.hub.force(phi, x)
        return grad_S * g, None, None, None, None, None, None
