"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws random numbers and nothing else: it holds none of the method's
arithmetic (no operator, no transform, no solver).  Both the HIP path and the CPU
oracle receive exactly the arrays produced here.

Workload shapes follow the lattices used for the honeycomb Hubbard model HMC
(Sec. 2 of the paper: largest lattice 20,808 sites = 2*102^2), and the field
distribution follows the Gaussian weight of the Hubbard field in the effective
Hamiltonian (eq. "hamiltonian"): with the phase written as e^{i phi} the field's
prior is N(0, sqrt(delta*U)), delta = beta/Nt.  The pseudofermion chi is drawn from
the density e^{-chi^dagger chi}, i.e. Re and Im parts ~ N(0, 1/2).  The heat-bath
vector rho (chi = M rho, Sec. 2) has the same density.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
import math

import numpy as np


@dataclass(frozen=True)
class Lattice:
    """One workload: an L x L honeycomb torus (2*L^2 sites) with Nt time slices."""
    name: str
    L: int
    Nt: int
    beta: float
    U: float
    kappa: float = 1.0
    nrhs: int = 1
    tol: float = 1e-12

    @property
    def V(self) -> int:
        return 2 * self.L * self.L

    @property
    def N(self) -> int:
        """Complex entries per vector per right-hand side."""
        return self.V * self.Nt

    @property
    def delta(self) -> float:
        return self.beta / self.Nt

    @property
    def phi_std(self) -> float:
        return math.sqrt(self.delta * self.U)

    def with_(self, **kw) -> "Lattice":
        return replace(self, **kw)


# The five workloads of the hot path, smallest first.
TINY = Lattice("L3_Nt8", L=3, Nt=8, beta=2.0, U=3.0, tol=1e-12)
SMALL = Lattice("L12_Nt32", L=12, Nt=32, beta=4.0, U=3.5, tol=1e-12)
DIFF = Lattice("L24_Nt64", L=24, Nt=64, beta=8.0, U=3.8, tol=1e-12)
PREC = Lattice("L51_Nt128", L=51, Nt=128, beta=8.0, U=3.85, tol=1e-10)
STRESS = Lattice("L102_Nt192_x4", L=102, Nt=192, beta=12.0, U=3.9, nrhs=4, tol=1e-10)
# An 18-site torus at the L=24 workload's time extent, small enough for dense algebra.
DIFF_SUB = Lattice("L3_Nt64", L=3, Nt=64, beta=8.0, U=3.8, tol=1e-12)

ALL = (TINY, SMALL, DIFF, PREC, STRESS)
BY_NAME = {w.name: w for w in ALL + (DIFF_SUB,)}


def draw_phi(w: Lattice, seed: int = 0, rng: np.random.Generator | None = None) -> np.ndarray:
    """Hubbard field, float64 [Nt, V] ~ N(0, sqrt(delta*U))."""
    rng = np.random.default_rng(seed) if rng is None else rng
    return rng.normal(0.0, w.phi_std, size=(w.Nt, w.V))


def draw_complex(w: Lattice, nrhs: int | None = None, rng: np.random.Generator | None = None,
                 seed: int = 0) -> np.ndarray:
    """Complex Gaussian with density e^{-z^dagger z}: complex128 [nrhs, Nt, V]."""
    rng = np.random.default_rng(seed) if rng is None else rng
    n = w.nrhs if nrhs is None else nrhs
    s = math.sqrt(0.5)
    re = rng.normal(0.0, s, size=(n, w.Nt, w.V))
    im = rng.normal(0.0, s, size=(n, w.Nt, w.V))
    return re + 1j * im


def draw_inputs(w: Lattice, seed: int = 0, nrhs: int | None = None):
    """(phi, chi) in the fixed draw order: phi first, then Re chi, then Im chi."""
    rng = np.random.default_rng(seed)
    phi = draw_phi(w, rng=rng)
    chi = draw_complex(w, nrhs=nrhs, rng=rng)
    return phi, chi


def draw_weak_field(w: Lattice, seed: int = 0, nrhs: int | None = None):
    """A labelled well-conditioned variant: the same draws with phi scaled by delta.

    This is the field normalisation in which the phase is e^{i delta phi} while phi
    keeps the prior std sqrt(delta*U); it gives a nearly free operator and is used
    only as a solver-speed workload, never as the headline input.
    """
    phi, chi = draw_inputs(w, seed=seed, nrhs=nrhs)
    return phi * w.delta, chi


def pick_entries(w: Lattice, count: int = 64, seed: int = 0) -> np.ndarray:
    """`count` distinct (t, x) field entries, as flat indices into [Nt, V]."""
    rng = np.random.default_rng(seed)
    return rng.choice(w.N, size=min(count, w.N), replace=False)


def draw_hmc_randoms(w: Lattice, n_traj: int, seed: int = 0, nrhs: int = 1):
    """Random numbers of n_traj HMC trajectories (Sec. 2): momenta pi ~ e^{-pi^2/2}
    (float64 [Nt, V]), heat-bath vectors rho ~ e^{-rho^dag rho} (complex128 [nrhs, Nt, V])
    and the Metropolis uniform u in [0, 1), in that order per trajectory."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_traj):
        pi = rng.normal(0.0, 1.0, size=(w.Nt, w.V))
        rho = draw_complex(w, nrhs=nrhs, rng=rng)
        u = float(rng.random())
        out.append((pi, rho, u))
    return out
