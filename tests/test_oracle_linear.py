"""Pins of the oracle's linear-form fermion matrix (eq. "ferm_op" as printed)."""
import numpy as np
import pytest

import oracle as O
from workloads import TINY, SMALL, draw_inputs, draw_complex, pick_entries
import closed_forms as CF


def _op(w):
    return O.LinearHubbardOperator(w.L, w.Nt, w.beta, w.kappa)


@pytest.mark.parametrize("L,Nt,beta", [(3, 4, 1.0), (3, 8, 2.0), (2, 6, 3.0), (4, 5, 1.5)])
def test_free_determinant_closed_form(L, Nt, beta):
    """phi = 0: time-Fourier (antiperiodic omega_n) and Bloch momentum k block-diagonalise M
    into [[e^{i w} - 1, -dk f], [-dk conj f, 1 - e^{-i w}]], so
    det M = prod_{k,n} -(4 sin^2(omega_n/2) + (delta kappa |f(k)|)^2)."""
    op = O.LinearHubbardOperator(L, Nt, beta)
    sign, ld = np.linalg.slogdet(op.dense_M(np.zeros((Nt, 2 * L * L))))
    om = (2 * np.arange(Nt) + 1) * np.pi / Nt
    f = np.abs(CF.f_of_k(L)).ravel()
    terms = -(4 * np.sin(om[:, None] / 2) ** 2 + (op.dk * f[None, :]) ** 2)
    assert abs(ld - np.log(np.abs(terms)).sum()) < 1e-11 * max(1, abs(ld))
    assert abs(sign - np.prod(np.sign(terms))) < 1e-10


def test_matrix_free_equals_dense_and_adjoint():
    w = TINY
    phi, v = draw_inputs(w, seed=2)
    u = draw_complex(w, seed=3)
    op = _op(w)
    M = op.dense_M(phi)
    np.testing.assert_allclose(op.apply_M(phi, v).ravel(), M @ v.ravel(), atol=1e-13)
    np.testing.assert_allclose(op.apply_Mdag(phi, v).ravel(), M.conj().T @ v.ravel(), atol=1e-13)
    a = np.vdot(u, op.apply_M(phi, v))
    b = np.vdot(op.apply_Mdag(phi, u), v)
    assert abs(a - b) < 1e-12 * abs(a)


def test_free_plane_wave_eigenvalues():
    """phi = 0 plane waves in time (antiperiodic omega) and space diagonalise the 2x2 block."""
    L, Nt, beta = 6, 8, 2.0
    op = O.LinearHubbardOperator(L, Nt, beta)
    rng = np.random.default_rng(3)
    for _ in range(4):
        n, m1, m2 = rng.integers(Nt), rng.integers(L), rng.integers(L)
        om = (2 * n + 1) * np.pi / Nt
        k1, k2 = 2 * np.pi * m1 / L, 2 * np.pi * m2 / L
        f = 1 + np.exp(-1j * k1) + np.exp(-1j * k2)
        blk = np.array([[np.exp(1j * om) - 1, -op.dk * f], [-op.dk * np.conj(f), 1 - np.exp(-1j * om)]])
        lam, vec = np.linalg.eig(blk)
        n1, n2 = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
        ph = np.exp(1j * (k1 * n1 + k2 * n2)).ravel()
        t = np.arange(Nt)
        for j in range(2):
            v = np.exp(1j * om * t)[:, None] * np.concatenate([vec[0, j] * ph, vec[1, j] * ph])[None, :]
            out = op.apply_M(np.zeros((Nt, 2 * L * L)), v[None])[0]
            np.testing.assert_allclose(out, lam[j] * v, atol=1e-12)


def test_force_definition_and_finite_differences():
    w = TINY
    phi, chi = draw_inputs(w)
    op = _op(w)
    x = O.dense_solve_op(op, phi, chi)
    g = O.force_linear(op, phi, x)
    gd = O.force_dense_linear(op, phi, x)
    assert np.linalg.norm(g - gd) <= 1e-12 * np.linalg.norm(gd)

    def S(p):
        return O.action(chi, O.dense_solve_op(op, p, chi))
    eps = 1e-6
    idx = pick_entries(w, 12)
    fd = []
    for i in idx:
        pp = phi.ravel().copy(); pp[i] += eps
        pm = phi.ravel().copy(); pm[i] -= eps
        fd.append((S(pp.reshape(phi.shape)) - S(pm.reshape(phi.shape))) / (2 * eps))
    assert np.linalg.norm(np.array(fd) - g.ravel()[idx]) <= 1e-6 * np.linalg.norm(g.ravel()[idx])


def test_heat_bath_and_cg():
    w = SMALL
    op = _op(w)
    phi = draw_inputs(w)[0]
    rho = draw_complex(w, seed=4)
    chi = op.apply_M(phi, rho)
    x, its, res = O.cg_solve(op, phi, chi, tol=1e-12)
    assert res[0] < 1e-11
    y = op.apply_Mdag(phi, x)
    assert np.linalg.norm(y - rho) <= 1e-8 * np.linalg.norm(rho)
