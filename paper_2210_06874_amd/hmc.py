"""Hybrid Monte Carlo trajectories of the Hubbard field on the device (Sec. 2).

Each trajectory: heat bath chi = M rho (rho ~ e^{-rho^dag rho}), momenta pi ~ e^{-pi^2/2},
molecular dynamics of H = pi^2/2 + phi^2/(2 delta U) + chi^dag (M M^dag)^{-1} chi with the
adjoint force, and acceptance with probability min(1, e^{-dH}).  The integrator is the
leapfrog or the second-order minimum-norm scheme of Omelyan, Mryglod and Folk (two force
evaluations per step, the last momentum update of a step merged with the first of the next).
The whole trajectory runs in the library (hub_trajectory): the random numbers are inputs,
every array operation is a library kernel, and the FP64 accept/reject decision is taken on
the two device-reduced energies.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch


@dataclass
class Trajectory:
    accepted: bool
    dH: float
    H0: float
    H1: float
    cg_iters: int
    n_forces: int


def trajectory(hub, phi: torch.Tensor, U: float, pi0: torch.Tensor, rho: torch.Tensor, u: float,
               n_md: int, eps: float, tol: float = 1e-10, prec: str = "mixed",
               max_iter: int = 200000, integrator: str = "leapfrog") -> Trajectory:
    """One HMC trajectory; `phi` (float64 [Nt, V] on the device) is updated in place and
    restored when the trajectory is rejected.  integrator: "leapfrog" (n_md + 1 force
    evaluations) or "omelyan" (2 n_md + 1)."""
    if integrator not in ("leapfrog", "omelyan"):
        raise ValueError(f"unknown integrator {integrator!r}")
    info = hub.trajectory(phi, pi0, rho, u, U, n_md, eps, integrator=integrator, tol=tol, prec=prec,
                          max_iter=max_iter)
    return Trajectory(bool(info.accepted), info.dH, info.H0, info.H1, info.cg_iters, info.n_forces)
