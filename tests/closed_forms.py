"""Closed forms of the free (phi = 0) and uniform-phase honeycomb operator.

These follow from Bloch's theorem on the L x L torus and are written here
independently of the oracle, which never uses momentum space:

* Sec. 1 (U = 0 limit): two bands +-kappa|f(k)| touching at the Dirac points,
  f(k) = 1 + e^{-i k1} + e^{-i k2}, k = 2 pi m / L.
* With antiperiodic time, the phi = 0 operator is diagonal in (Matsubara
  frequency omega_n = (2n+1) pi / Nt, momentum k, band +-):
  eigenvalue 1 - e^{-i omega_n} e^{delta eps}, eps = +-kappa|f(k)|.
* log det M(phi=0) = sum_{k,+-} log(1 + e^{+-beta kappa |f(k)|}).
"""
import numpy as np


def momenta(L):
    k = 2.0 * np.pi * np.arange(L) / L
    return np.meshgrid(k, k, indexing="ij")       # (k1, k2) matching (n1, n2)


def f_of_k(L):
    k1, k2 = momenta(L)
    return 1.0 + np.exp(-1j * k1) + np.exp(-1j * k2)


def free_log_det(L, beta, kappa=1.0, total_phase=0.0):
    """log det M for phi_{t,x} = c_t with sum_t c_t = total_phase (complex log)."""
    a = np.abs(f_of_k(L)).ravel()
    z = np.exp(1j * total_phase)
    terms = np.concatenate([np.log(1 + z * np.exp(beta * kappa * a)),
                            np.log(1 + z * np.exp(-beta * kappa * a))])
    return terms.sum()


def plane_wave(L, Nt, n, m1, m2, band):
    """Eigenvector of the phi = 0 operator: time frequency index n, momentum (m1, m2),
    band +1/-1.  Returns (vector [Nt, 2L^2], energy eps/kappa, omega)."""
    k1 = 2 * np.pi * m1 / L
    k2 = 2 * np.pi * m2 / L
    f = 1 + np.exp(-1j * k1) + np.exp(-1j * k2)
    af = abs(f)
    if af < 1e-12:          # Dirac point: K(k) = 0, any spinor is an eigenvector
        ua, ub = 1.0, band * 1.0
        eps = 0.0
    else:
        ua, ub = f / af, band * 1.0
        eps = band * af
    n1, n2 = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    # angles reduced with integer arithmetic, so every phase is accurate to ~1e-16
    ph = np.exp(2j * np.pi * ((m1 * n1 + m2 * n2) % L) / L).ravel()
    spatial = np.concatenate([ua * ph, ub * ph]) / np.sqrt(2 * L * L)
    omega = (2 * n + 1) * np.pi / Nt
    t = np.arange(Nt)
    v = np.exp(1j * np.pi * (((2 * n + 1) * t) % (2 * Nt)) / Nt)[:, None] * spatial[None, :] / np.sqrt(Nt)
    return v, eps, omega


def free_M_eigenvalue(eps_over_kappa, omega, delta, kappa=1.0):
    return 1.0 - np.exp(-1j * omega) * np.exp(delta * kappa * eps_over_kappa)
