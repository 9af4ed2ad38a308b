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


# ----------------------------------------------------------------------------- phi != 0 pins
def momentum_block(L, Nt, dk, c, m1, m2):
    """The linear operator of eq. "ferm_op" at a field phi_{t,x} = c_t (the same on every site)
    restricted to one spatial momentum k = 2 pi (m1, m2) / L, written out from the equation
    with time as an explicit index: a 2 Nt x 2 Nt matrix acting on (a_0..a_{Nt-1}, b_0..b_{Nt-1}),
    the amplitudes of the plane wave e^{i k.n} on sublattices A and B.  The hopping sends a
    plane wave on B to f(k) times it on A, and one on A to conj f(k) times it on B, with
    f(k) = 1 + e^{-i k1} + e^{-i k2} (A(n) bonded to B(n), B(n - e1), B(n - e2));
    the time hop across the wrap carries the antiperiodic -1."""
    f = 1 + np.exp(-2j * np.pi * m1 / L) + np.exp(-2j * np.pi * m2 / L)
    sign = lambda t: -1.0 if t % Nt == 0 else 1.0           # B_t: -1 on the wrap
    blk = np.zeros((2 * Nt, 2 * Nt), dtype=complex)
    for t in range(Nt):
        a, b = t, Nt + t
        # A rows: B_{t+1} a_{t+1} - e^{i c_t} a_t - dk f b_t
        blk[a, (t + 1) % Nt] += sign(t + 1)
        blk[a, t] -= np.exp(1j * c[t])
        blk[a, Nt + t] -= dk * f
        # B rows: b_t - B_t e^{-i c_t} b_{t-1} - dk conj(f) a_t
        blk[b, Nt + t] += 1.0
        blk[b, Nt + (t - 1) % Nt] -= sign(t) * np.exp(-1j * c[t])
        blk[b, t] -= dk * np.conj(f)
    return blk


def _plane(L, m1, m2):
    n1, n2 = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    return np.exp(2j * np.pi * ((m1 * n1 + m2 * n2) % L) / L).ravel()


def check_uniform_field_momentum_blocks(cls=None, L=3, Nt=6, beta=2.0, seed=5):
    """phi_{t,x} = c_t with c_t varying in time: on every plane wave in space M and M^dag act as
    the momentum block and its adjoint, and log det M is the sum of the blocks' log dets."""
    op = (cls or O.LinearHubbardOperator)(L, Nt, beta)
    rng = np.random.default_rng(seed)
    c = rng.uniform(-np.pi, np.pi, size=Nt)
    phi = np.repeat(c[:, None], op.V, axis=1)
    ok = True
    ld_sum, ph_sum = 0.0, 0.0
    for m1 in range(L):
        for m2 in range(L):
            blk = momentum_block(L, Nt, op.dk, c, m1, m2)
            s, ld = np.linalg.slogdet(blk)
            ld_sum += ld
            ph_sum += np.angle(s)
            ab = rng.normal(size=2 * Nt) + 1j * rng.normal(size=2 * Nt)
            pw = _plane(L, m1, m2)
            v = np.concatenate([ab[:Nt, None] * pw[None], ab[Nt:, None] * pw[None]], axis=1)
            for out, mat in ((op.apply_M(phi, v[None])[0], blk), (op.apply_Mdag(phi, v[None])[0], blk.conj().T)):
                y = mat @ ab
                ref = np.concatenate([y[:Nt, None] * pw[None], y[Nt:, None] * pw[None]], axis=1)
                ok &= np.abs(out - ref).max() < 1e-12 * np.abs(ref).max()
    s, ld = np.linalg.slogdet(op.dense_M(phi))
    ok &= abs(ld - ld_sum) < 1e-11 * max(1.0, abs(ld))
    ok &= abs(s - np.exp(1j * ph_sum)) < 1e-10
    return bool(ok)


def check_single_site_phase_determinant(cls=None, L=2, Nt=5, beta=1.5):
    """A field on one site only changes one entry of M (eq. "ferm_op": the A-site diagonal
    -e^{i phi_{t,x}}, or the B-site hop -B_t e^{-i phi_{t,x}} from slice t-1), so by the
    determinant lemma det M[phi] = det M[0] (1 + D (M[0]^{-1})_{c,r}) with D the change of
    entry (r, c).  M[0] is pinned by the free determinant and the plane-wave eigenvalues."""
    op = (cls or O.LinearHubbardOperator)(L, Nt, beta)
    M0 = op.dense_M(np.zeros((Nt, op.V)))
    G = np.linalg.inv(M0)
    s0, ld0 = np.linalg.slogdet(M0)
    ok = True
    for (t, x, val) in [(2, 1, 0.7), (0, op.V - 1, -1.1), (Nt - 1, 0, 2.3), (3, op.nA, 0.4)]:
        phi = np.zeros((Nt, op.V))
        phi[t, x] = val
        r = t * op.V + x
        if x < op.nA:
            c, D = r, -(np.exp(1j * val) - 1.0)
        else:
            Bt = -1.0 if t == 0 else 1.0
            c, D = ((t - 1) % Nt) * op.V + x, -Bt * (np.exp(-1j * val) - 1.0)
        s, ld = np.linalg.slogdet(op.dense_M(phi))
        want = s0 * np.exp(ld0) * (1.0 + D * G[c, r])
        ok &= abs(s * np.exp(ld) - want) < 1e-10 * abs(want)
    return bool(ok)


def test_uniform_field_momentum_blocks():
    """A fixed fact at phi != 0 that depends on where and with which sign every phase enters."""
    assert check_uniform_field_momentum_blocks()
    assert check_uniform_field_momentum_blocks(L=4, Nt=5, beta=3.0, seed=7)


def test_single_site_phase_determinant_lemma():
    assert check_single_site_phase_determinant()
    assert check_single_site_phase_determinant(L=3, Nt=4, beta=2.0)
