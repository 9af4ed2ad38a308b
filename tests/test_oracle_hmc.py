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


@pytest.mark.parametrize("integrator", ["leapfrog", "omelyan"])
@pytest.mark.parametrize("form", ["exp", "linear"])
def test_reversibility(form, integrator):
    """Integrate forward, flip the momentum, integrate back: the field returns."""
    w, op, phi, pi, rho, u = _setup(form)
    chi = op.apply_M(phi, rho)
    phi1, pi1, dH, _, _ = OH.trajectory(op, w.U, phi, pi, rho, u, n_md=6, eps=0.05, integrator=integrator)
    # backwards with the same chi: a trajectory from (phi1, -pi1) whose heat bath gives chi
    rho_back = np.linalg.solve(op.dense_M(phi1), chi.ravel()).reshape(rho.shape)
    phi2, pi2, dH2, _, _ = OH.trajectory(op, w.U, phi1, -pi1, rho_back, u, n_md=6, eps=0.05,
                                         integrator=integrator)
    np.testing.assert_allclose(phi2, phi, atol=1e-9)
    np.testing.assert_allclose(-pi2, pi, atol=1e-9)
    assert abs(dH + dH2) < 1e-9


@pytest.mark.parametrize("integrator", ["leapfrog", "omelyan"])
@pytest.mark.parametrize("form", ["exp", "linear"])
def test_energy_error_is_second_order(form, integrator):
    """Both integrators: dH(eps) ~ eps^2 at fixed trajectory length, so halving eps quarters
    dH.  A force that is not the gradient of H breaks this scaling.  (The linear form's
    fourth-order term is larger on this field: its asymptotic regime starts at a shorter
    trajectory.)"""
    w, op, phi, pi, rho, u = _setup(form)
    dh = []
    T = 0.8 if form == "exp" else 0.4
    steps = (16, 32, 64) if integrator == "leapfrog" else (8, 16, 32)
    for n in steps:
        eps = T / n
        dh.append(abs(OH.trajectory(op, w.U, phi, pi, rho, u, n_md=n, eps=eps, integrator=integrator)[2]))
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


def test_omelyan_at_a_quarter_is_two_leapfrog_steps(monkeypatch):
    """With lambda = 1/4 one Omelyan step of eps is exactly two leapfrog steps of eps/2
    (the kicks eps/4, eps/2, eps/4 around two half drifts): the step sequence is pinned
    against the leapfrog independently of the value of lambda."""
    w, op, phi, pi, rho, u = _setup("exp")
    monkeypatch.setattr(OH, "OMELYAN_LAMBDA", 0.25)
    a = OH.trajectory(op, w.U, phi, pi, rho, u, n_md=5, eps=0.08, integrator="omelyan")
    b = OH.trajectory(op, w.U, phi, pi, rho, u, n_md=10, eps=0.04)
    np.testing.assert_allclose(a[0], b[0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(a[1], b[1], rtol=0, atol=1e-12)
    assert abs(a[2] - b[2]) < 1e-11


def test_omelyan_lambda_is_the_minimum_norm_choice():
    """The two-stage scheme's third-order error has coefficients (6 l^2 - 6 l + 1)/12 and
    (1 - 6 l)/24 on its two nested commutators; the integrator's lambda minimises their
    Euclidean norm."""
    from scipy.optimize import minimize_scalar
    f = lambda l: ((6 * l * l - 6 * l + 1) / 12) ** 2 + ((1 - 6 * l) / 24) ** 2
    best = minimize_scalar(f, bounds=(0.0, 0.5), method="bounded", options={"xatol": 1e-13}).x
    assert abs(best - OH.OMELYAN_LAMBDA) < 1e-8


def test_unknown_integrator_is_refused():
    w, op, phi, pi, rho, u = _setup("exp")
    with pytest.raises(ValueError):
        OH.trajectory(op, w.U, phi, pi, rho, u, n_md=2, eps=0.1, integrator="rk4")


def _free_field_chain(n=300, seed=5):
    """A chain with rho = 0, hence chi = 0 and no fermion action: the Hamiltonian's field part
    alone, pi^2/2 + phi^2/(2 delta U), a harmonic oscillator of frequency 1/sqrt(delta U).  Each
    trajectory runs a quarter period, which maps the refreshed momentum to a fresh, independent
    field.  2 x 2 torus, N_t = 4, beta = 1, U = 2 (delta U = 0.5).  Returns the mean of phi^2 over
    every entry of every field and its standard error from 20 batch means."""
    w = Lattice("L2_Nt4", 2, 4, 1.0, 2.0)
    op = O.HubbardOperator(w.L, w.Nt, w.beta, w.kappa)
    n_md = 16
    eps = 0.5 * math.pi * math.sqrt(w.delta * w.U) / n_md
    phi = np.zeros((w.Nt, w.V))
    sq = []
    for pi, rho, u in draw_hmc_randoms(w, n, seed=seed):
        phi = OH.trajectory(op, w.U, phi, pi, 0.0 * rho, u, n_md=n_md, eps=eps)[4]
        sq.append(np.mean(phi * phi))
    sq = np.array(sq)
    batches = sq.reshape(20, -1).mean(axis=1)
    return w, sq.mean(), batches.std() / math.sqrt(20)


def test_field_prior_variance_is_delta_u():
    """The Gaussian term of eq. "hamiltonian" (phi^2/(2 delta U) with phi = delta times the
    paper's field) fixes the field's variance without fermions: <phi^2> = delta U, the prior
    std sqrt(delta U) of the workloads."""
    w, m, se = _free_field_chain()
    assert se < 0.02 * w.delta * w.U and abs(m - w.delta * w.U) < 5 * se, (m, se, w.delta * w.U)


def test_field_prior_variance_detects_a_wrong_normalisation(monkeypatch):
    """Planted consistently in the Hamiltonian and its force: phi^2/(2U) instead of
    phi^2/(2 delta U).  The dynamics stay reversible and energy-conserving, but the chain's
    <phi^2> becomes U, not delta U."""
    def ham(op, U, phi, pi, chi, x):
        return 0.5 * float(np.sum(pi * pi)) + float(np.sum(phi * phi)) / (2.0 * U) + O.action(chi, x)

    def tot(op, U, phi, x):
        return phi / U + O.force(op, phi, x)
    monkeypatch.setattr(OH, "hamiltonian", ham)
    monkeypatch.setattr(OH, "total_force", tot)
    w, m, se = _free_field_chain()
    assert abs(m - w.delta * w.U) > 5 * se, (m, se)
