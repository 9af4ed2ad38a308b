"""Hybrid Monte Carlo trajectories of the Hubbard field on the device (Sec. 2).

Each trajectory: heat bath chi = M rho (rho ~ e^{-rho^dag rho}), momenta pi ~ e^{-pi^2/2},
molecular dynamics of H = pi^2/2 + phi^2/(2 delta U) + chi^dag (M M^dag)^{-1} chi with the
adjoint force, and acceptance with probability min(1, e^{-dH}).  The integrator is the
leapfrog or the second-order minimum-norm scheme of Omelyan, Mryglod and Folk (two force
evaluations per step, the last momentum update of a step merged with the first of the next).  The random
numbers are inputs; every array operation runs in the library's kernels (operator, CG,
force, MD update, energies); the host only sequences the calls and takes the FP64
accept/reject decision from the two device-reduced energies.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch


@dataclass
class Trajectory:
    accepted: bool
    dH: float
    H0: float
    H1: float
    cg_iters: list
    n_forces: int


OMELYAN_LAMBDA = 0.1931833275037836   # minimum-norm coefficient of the two-stage scheme


def trajectory(hub, phi: torch.Tensor, U: float, pi0: torch.Tensor, rho: torch.Tensor, u: float,
               n_md: int, eps: float, tol: float = 1e-10, prec: str = "mixed",
               max_iter: int = 200000, integrator: str = "leapfrog") -> Trajectory:
    """One HMC trajectory; `phi` (float64 [Nt, V] on the device) is updated in place and
    restored when the trajectory is rejected.  integrator: "leapfrog" (n_md + 1 force
    evaluations) or "omelyan" (2 n_md + 1)."""
    if integrator not in ("leapfrog", "omelyan"):
        raise ValueError(f"unknown integrator {integrator!r}")
    phi_start = phi.clone()
    pi = pi0.clone()
    chi = hub.apply_M(phi, rho)
    iters = []

    def solve(x0):
        res = hub.cg_solve(phi, chi, tol=tol, prec=prec, max_iter=max_iter, x0=x0)
        iters.append(res.iters[0] if len(res.iters) == 1 else list(res.iters))
        return res.x

    x = solve(None)
    H0 = hub.boson_energy(phi, pi, U).item() + hub.action(chi, x).item()
    g = hub.force(phi, x)
    if integrator == "leapfrog":
        hub.md_update(phi, pi, g, U, 0.5 * eps, eps)
        for s in range(1, n_md + 1):
            x = solve(x)
            hub.force(phi, x, out=g)
            if s < n_md:
                hub.md_update(phi, pi, g, U, eps, eps)
            else:
                hub.md_update(phi, pi, g, U, 0.5 * eps, 0.0)
    else:
        lam = OMELYAN_LAMBDA
        hub.md_update(phi, pi, g, U, lam * eps, 0.5 * eps)
        for s in range(1, n_md + 1):
            x = solve(x)
            hub.force(phi, x, out=g)
            hub.md_update(phi, pi, g, U, (1.0 - 2.0 * lam) * eps, 0.5 * eps)
            x = solve(x)
            hub.force(phi, x, out=g)
            if s < n_md:
                hub.md_update(phi, pi, g, U, 2.0 * lam * eps, 0.5 * eps)
            else:
                hub.md_update(phi, pi, g, U, lam * eps, 0.0)
    H1 = hub.boson_energy(phi, pi, U).item() + hub.action(chi, x).item()
    dH = H1 - H0
    accepted = dH <= 0.0 or u < math.exp(-dH)
    if not accepted:
        phi.copy_(phi_start)
    return Trajectory(bool(accepted), dH, H0, H1, iters, n_md + 1 if integrator == "leapfrog" else 2 * n_md + 1)
