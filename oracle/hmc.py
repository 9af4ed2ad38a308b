"""FP64 CPU oracle of one HMC trajectory (Sec. 2).  TEST INFRASTRUCTURE ONLY.

Hamiltonian (eq. "hamiltonian", with phi = delta * the paper's field):
    H = sum pi^2/2 + sum phi^2/(2 delta U) + chi^dag (M M^dag)^{-1} chi.
The trajectory draws nothing itself: the momenta pi0, the heat-bath vector rho
(chi = M rho) and the Metropolis uniform u are inputs.  Molecular dynamics is the
leapfrog (half momentum step, alternating full steps, half momentum step) or the
second-order minimum-norm integrator of Omelyan, Mryglod and Folk (per step: momentum
by lambda*eps, field by eps/2, momentum by (1 - 2 lambda)*eps, field by eps/2, momentum
by lambda*eps); the trajectory is accepted with probability min(1, e^{-dH}).  The operator may be either
form of the fermion matrix (HubbardOperator or LinearHubbardOperator); the force is the
one of that form.  The normalisation of the Gaussian term is pinned by a chain without
fermions (rho = 0), whose field variance must be delta*U (tests/test_oracle_hmc.py).
"""
from __future__ import annotations

import math

import numpy as np

from .hubbard import (HubbardOperator, LinearHubbardOperator, cg_solve, dense_solve, dense_solve_op, action,
                      force, force_linear)


def _solve(op, phi, chi, tol, dense):
    if dense:
        return dense_solve_op(op, phi, chi) if isinstance(op, LinearHubbardOperator) else dense_solve(op, phi, chi)
    x, _, _ = cg_solve(op, phi, chi, tol=tol)
    return x


def hamiltonian(op: HubbardOperator, U: float, phi, pi, chi, x) -> float:
    return 0.5 * float(np.sum(pi * pi)) + float(np.sum(phi * phi)) / (2.0 * op.delta * U) + action(chi, x)


def total_force(op: HubbardOperator, U: float, phi, x) -> np.ndarray:
    """dH/dphi = phi/(delta U) + dS_f/dphi."""
    g = force_linear(op, phi, x) if isinstance(op, LinearHubbardOperator) else force(op, phi, x)
    return phi / (op.delta * U) + g


# the minimum-norm choice of the Omelyan-Mryglod-Folk second-order integrator
OMELYAN_LAMBDA = 0.1931833275037836


def trajectory(op: HubbardOperator, U: float, phi0, pi0, rho, u: float, n_md: int, eps: float,
               tol: float = 1e-12, dense: bool | None = None, integrator: str = "leapfrog"):
    """Returns (phi_end, pi_end, dH, accepted, phi_out) with phi_out = phi_end if accepted
    else phi0.  integrator: "leapfrog" (n_md + 1 force evaluations) or "omelyan"
    (2 n_md + 1)."""
    if dense is None:
        dense = op.N <= 2000
    phi = np.array(phi0, dtype=float)
    pi = np.array(pi0, dtype=float)
    chi = op.apply_M(phi, rho)
    x = _solve(op, phi, chi, tol, dense)
    H0 = hamiltonian(op, U, phi, pi, chi, x)
    if integrator == "leapfrog":
        pi = pi - 0.5 * eps * total_force(op, U, phi, x)
        for s in range(n_md):
            phi = phi + eps * pi
            x = _solve(op, phi, chi, tol, dense)
            step = eps if s < n_md - 1 else 0.5 * eps
            pi = pi - step * total_force(op, U, phi, x)
    elif integrator == "omelyan":
        lam = OMELYAN_LAMBDA
        for s in range(n_md):
            pi = pi - lam * eps * total_force(op, U, phi, x)
            phi = phi + 0.5 * eps * pi
            x = _solve(op, phi, chi, tol, dense)
            pi = pi - (1.0 - 2.0 * lam) * eps * total_force(op, U, phi, x)
            phi = phi + 0.5 * eps * pi
            x = _solve(op, phi, chi, tol, dense)
            pi = pi - lam * eps * total_force(op, U, phi, x)
    else:
        raise ValueError(f"unknown integrator {integrator!r}")
    H1 = hamiltonian(op, U, phi, pi, chi, x)
    dH = H1 - H0
    accepted = bool(dH <= 0.0 or u < math.exp(-dH))
    return phi, pi, dH, accepted, (phi if accepted else np.array(phi0, dtype=float))
