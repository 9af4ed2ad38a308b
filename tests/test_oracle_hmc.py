"""Pins of the oracle HMC trajectory: time reversibility, second-order energy error of
the leapfrog (which also pins the force against the Hamiltonian), the heat bath, and the
equilibrium identity <e^{-dH}> = 1 of a chain of trajectories."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import hmc as OH
from workloads import TINY, Lattice, draw_weak_field, draw_hmc_randoms


def _setup(form="exp"):
    # a well-conditioned starting field (prior draws scaled by delta), where the leapfrog
    # is in its asymptotic regime at these step sizes
    w = TINY
    cls = O.LinearHubbardOperator if form == "linear" else O.HubbardOperator
    op = cls(w.L, w.Nt, w.beta, w.kappa)
    phi = draw_weak_field(w)[0]
    (pi, rho, u), = draw_hmc_randoms(w, 1, seed=3)
    return w, op, phi, pi, rho, u


@pytest.mark.parametrize("form", ["exp", "linear"])
def test_reversibility(form):
    """Integrate forward, flip the momentum, integrate back: the field returns."""
    w, op, phi, pi, rho, u = _setup(form)
    chi = op.apply_M(phi, rho)
    phi1, pi1, dH, _, _ = OH.trajectory(op, w.U, phi, pi, rho, u, n_md=6, eps=0.05)
    # backwards with the same chi: a trajectory from (phi1, -pi1) whose heat bath gives chi
    rho_back = np.linalg.solve(op.dense_M(phi1), chi.ravel()).reshape(rho.shape)
    phi2, pi2, dH2, _, _ = OH.trajectory(op, w.U, phi1, -pi1, rho_back, u, n_md=6, eps=0.05)
    np.testing.assert_allclose(phi2, phi, atol=1e-9)
    np.testing.assert_allclose(-pi2, pi, atol=1e-9)
    assert abs(dH + dH2) < 1e-9


@pytest.mark.parametrize("form", ["exp", "linear"])
def test_energy_error_is_second_order(form):
    """Leapfrog: dH(eps) ~ eps^2 at fixed trajectory length, so halving eps quarters dH.
    A force that is not the gradient of H breaks this scaling.  (The linear form's
    fourth-order term is larger on this field: its asymptotic regime starts at a shorter
    trajectory.)"""
    w, op, phi, pi, rho, u = _setup(form)
    dh = []
    T = 0.8 if form == "exp" else 0.4
    for n in (16, 32, 64):
        eps = T / n
        dh.append(abs(OH.trajectory(op, w.U, phi, pi, rho, u, n_md=n, eps=eps)[2]))
    r1, r2 = dh[0] / dh[1], dh[1] / dh[2]
    assert 3.3 < r1 < 4.7 and 3.6 < r2 < 4.4, (dh, r1, r2)


@pytest.mark.parametrize("form", ["exp", "linear"])
def test_heat_bath_initial_action(form):
    """Sec. 2: chi = M rho gives chi^dag (M M^dag)^{-1} chi = rho^dag rho."""
    w, op, phi, pi, rho, u = _setup(form)
    chi = op.apply_M(phi, rho)
    x = O.dense_solve_op(op, phi, chi)
    assert abs(O.action(chi, x) - np.vdot(rho, rho).real) < 1e-9 * np.vdot(rho, rho).real


def test_metropolis_decision():
    w, op, phi, pi, rho, u = _setup()
    phi1, pi1, dH, acc, out = OH.trajectory(op, w.U, phi, pi, rho, u, n_md=4, eps=0.1)
    assert acc == (dH <= 0 or u < np.exp(-dH))
    np.testing.assert_array_equal(out, phi1 if acc else phi)


def _creutz_chain(form, rho_scale=1.0, n=2000, burn=200):
    """A Markov chain of trajectories on a 2 x 2 torus (N_t = 4, beta = 1, U = 2) from phi = 0:
    e^{-dH} of every trajectory after the burn-in, and the standard error from 20 batch means."""
    w = Lattice("L2_Nt4", 2, 4, 1.0, 2.0)
    cls = O.LinearHubbardOperator if form == "linear" else O.HubbardOperator
    op = cls(w.L, w.Nt, w.beta, w.kappa)
    phi = np.zeros((w.Nt, w.V))
    ex = []
    for k, (pi, rho, u) in enumerate(draw_hmc_randoms(w, n, seed=1)):
        _, _, dH, _, phi = OH.trajectory(op, w.U, phi, pi, rho_scale * rho, u, n_md=20, eps=0.05)
        if k >= burn:
            ex.append(math.exp(-dH) if dH > -700 else math.inf)
    ex = np.array(ex)
    batches = ex[: len(ex) // 20 * 20].reshape(20, -1).mean(axis=1)
    return ex.mean(), batches.std() / math.sqrt(20)


@pytest.mark.parametrize("form", ["exp", "linear"])
def test_creutz_equality(form):
    """In equilibrium <e^{-dH}> = 1 for a reversible, area-preserving integrator, whatever its
    step size: the chain (momentum refresh, heat bath chi = M rho, leapfrog, Metropolis) samples
    the distribution its Hamiltonian defines.  A trajectory that meets a near-zero of det M
    can blow up; it is rejected and contributes e^{-dH} ~ 0, as it should."""
    m, se = _creutz_chain(form)
    assert se < 0.01 and abs(m - 1.0) < 5 * se, (m, se)


def test_creutz_equality_detects_a_wrong_heat_bath():
    """rho drawn with twice the variance of e^{-rho^dag rho}: the chain no longer samples the
    Hamiltonian's distribution and <e^{-dH}> leaves 1 (by about 8 standard errors here)."""
    m, se = _creutz_chain("exp", rho_scale=math.sqrt(2.0))
    assert abs(m - 1.0) > 5 * se, (m, se)
