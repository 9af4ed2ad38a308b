"""The pseudofermion action as a differentiable function of the Hubbard field and chi.

S[phi, chi] = chi^dag (M M^dag)^{-1} chi   (Sec. 2, eq. "hamiltonian")

forward:  x = CG(phi, chi) on the device, S = Re chi^dag x.
backward: dS/dphi from the adjoint force kernel, which reuses the CG solution x
          and recomputes E x per slice; nothing is stored per slice.
          For chi (complex), torch's convention for a real function gives 2 dS/dchi^* = 2 x,
          since M M^dag is Hermitian.
"""
from __future__ import annotations

import torch


class PseudofermionAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, chi, hub, tol=1e-10, prec="fp64", max_iter=100000, reliable_every=50):
        res = hub.cg_solve(phi, chi, tol=tol, max_iter=max_iter, prec=prec, reliable_every=reliable_every)
        S = hub.action(chi, res.x)
        ctx.hub = hub
        ctx.chi_shape = chi.shape
        ctx.save_for_backward(phi, res.x)
        ctx.cg = res
        return S

    @staticmethod
    def backward(ctx, grad_S):
        phi, x = ctx.saved_tensors
        g_phi = grad_S * ctx.hub.force(phi, x) if ctx.needs_input_grad[0] else None
        g_chi = (2.0 * grad_S) * x.reshape(ctx.chi_shape) if ctx.needs_input_grad[1] else None
        return g_phi, g_chi, None, None, None, None, None
