"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

None of these retypes the oracle's own formulas: each compares the oracle with a
closed form, a library routine reached by a different route, an algebraic
identity, or brute force.  See tests/test_oracle_mutants.py for the check that
plausible mistakes in the oracle make at least one pin fail.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle as O
from workloads import TINY, SMALL, DIFF_SUB, draw_inputs, draw_complex, pick_entries
import closed_forms as CF

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _op(w, **kw):
    return O.HubbardOperator(w.L, w.Nt, w.beta, w.kappa, **kw)


# ----------------------------------------------------------------------------- geometry
@pytest.mark.parametrize("L", [1, 2, 3, 4, 6, 7])
def test_hopping_spectrum_is_two_bands(L):
    """Sec. 1 (U = 0): the spectrum of K is {+|f(k)|, -|f(k)|} over the L^2 momenta."""
    K = O.hopping_matrix(L)
    lam = np.sort(np.linalg.eigvalsh(K))
    a = np.abs(CF.f_of_k(L)).ravel()
    ref = np.sort(np.concatenate([a, -a]))
    np.testing.assert_allclose(lam, ref, atol=1e-12)


@pytest.mark.parametrize("L", [2, 3, 5])
def test_hopping_bipartite_degree_three(L):
    """Fig. "honeycomb_lattice": every site has 3 neighbours, all on the other sublattice."""
    K = O.hopping_matrix(L)
    V = 2 * L * L
    h = L * L
    assert np.all(K[:h, :h] == 0) and np.all(K[h:, h:] == 0)
    np.testing.assert_array_equal(K, K.T)
    np.testing.assert_array_equal(K.sum(axis=1), np.full(V, 3.0))
    # sigma K sigma = -K (bipartite), sigma = diag(+1_A, -1_B)
    sig = np.concatenate([np.ones(h), -np.ones(h)])
    np.testing.assert_array_equal(sig[:, None] * K * sig[None, :], -K)


def _figure_geometry():
    """tests/golden/honeycomb_figure_geometry.txt: the Sec. 1 figure's own coordinates."""
    import os
    vals, bonds = {}, []
    with open(os.path.join(os.path.dirname(__file__), "golden", "honeycomb_figure_geometry.txt")) as f:
        for line in f:
            parts = line.split()
            if not parts or parts[0].startswith("#"):
                continue
            if parts[0] == "bond":
                bonds.append(np.array([float(parts[1]), float(parts[2])]))
            else:
                vals[parts[0]] = float(parts[1])
    return vals, bonds


def test_hopping_brute_force_from_the_figure_L3():
    """Brute force from the paper's drawing (Sec. 1 figure, golden fixture): place A sites on the
    figure's triangular lattice and B sites along its horizontal bond, link sites at unit
    distance on the L = 3 torus, and compare with the oracle's K.  The figure's other two
    bond vectors are the oracle's B(n - e2) and B(n - e1) neighbours."""
    L = 3
    g, bonds = _figure_geometry()
    cs, rs, sh = g["column_spacing"], g["row_spacing"], g["odd_column_shift"]
    a1 = np.array([cs, sh])             # A(column 1, row 0) - A(0, 0)
    a2 = np.array([cs, sh - rs])        # A(column 1, row -1) - A(0, 0)
    b0 = bonds[0]                       # B(n) = A(n) + the horizontal bond
    assert len(bonds) == 3 and all(abs(np.linalg.norm(b) - 1.0) < 1e-3 for b in bonds)
    np.testing.assert_allclose(bonds[1], -a2 + b0, atol=2e-3)     # B(n - e2)
    np.testing.assert_allclose(bonds[2], -a1 + b0, atol=2e-3)     # B(n - e1)
    pos = {}
    for s in (0, 1):
        for n1 in range(L):
            for n2 in range(L):
                pos[O.site_index(L, s, n1, n2)] = n1 * a1 + n2 * a2 + (b0 if s else 0.0)
    # torus: distance minimised over periodic images; the next-nearest distance is sqrt(3)
    V = 2 * L * L
    K = np.zeros((V, V))
    for x in range(V):
        for y in range(V):
            d = min(np.linalg.norm(pos[x] - pos[y] + i * L * a1 + j * L * a2)
                    for i in (-1, 0, 1) for j in (-1, 0, 1))
            if abs(d - 1.0) < 0.02:
                K[x, y] = 1.0
    np.testing.assert_array_equal(K, O.hopping_matrix(L))


@pytest.mark.parametrize("L,dk", [(3, 0.25), (4, 0.125), (6, 0.0625)])
def test_hopping_exponential_matches_expm(L, dk):
    """exp(delta kappa K) from eigh equals scipy.linalg.expm (Pade) and the Krylov route."""
    E = O.hopping_exponential(L, dk)
    np.testing.assert_allclose(E, scipy.linalg.expm(dk * O.hopping_matrix(L)), atol=2e-15, rtol=0)
    op = O.HubbardOperator(L, 2, 2 * dk, 1.0, mode="expm")
    v = np.random.default_rng(3).normal(size=(5, 2 * L * L)) + 0j
    np.testing.assert_allclose(op.apply_E(v), v @ E.T, atol=1e-14, rtol=0)


# ----------------------------------------------------------------------------- determinant
@pytest.mark.parametrize("L,Nt,beta", [(3, 8, 2.0), (3, 64, 8.0), (2, 5, 1.0), (4, 6, 3.0), (1, 3, 1.5)])
def test_free_log_det_closed_form(L, Nt, beta):
    """Sec. 1/2: at U = 0 (phi = 0), det M = prod_{k,+-} (1 + e^{+-beta kappa |f(k)|})."""
    op = O.HubbardOperator(L, Nt, beta)
    sign, ld = np.linalg.slogdet(op.dense_M(np.zeros((Nt, 2 * L * L))))
    ref = CF.free_log_det(L, beta)
    assert abs(ld - ref.real) < 1e-12 * max(1.0, abs(ref))
    assert abs(sign - 1) < 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_uniform_phase_log_det(seed):
    """phi_{t,x} = c_t (slice-uniform): det M = prod_{k,+-}(1 + e^{i sum c} e^{+-beta kappa |f|})."""
    L, Nt, beta = 3, 8, 2.0
    c = np.random.default_rng(seed).normal(0, 0.7, size=Nt)
    op = O.HubbardOperator(L, Nt, beta)
    det = np.linalg.det(op.dense_M(np.repeat(c[:, None], 2 * L * L, axis=1)))
    ref = np.exp(CF.free_log_det(L, beta, total_phase=c.sum()))
    assert abs(det - ref) < 1e-11 * abs(ref)


def test_log_det_equals_transfer_product():
    """Block-cyclic determinant: det M = det(1 + E D_{Nt-1} ... E D_0) (antiperiodic wrap)."""
    w = TINY
    phi, _ = draw_inputs(w)
    op = _op(w)
    P = np.eye(w.V, dtype=complex)
    for t in range(w.Nt):
        P = op.E @ (np.exp(1j * phi[t])[:, None] * P)
    s1, l1 = np.linalg.slogdet(op.dense_M(phi))
    s2, l2 = np.linalg.slogdet(np.eye(w.V) + P)
    assert abs(l1 - l2) < 1e-11 and abs(s1 - s2) < 1e-11


def test_weight_is_positive_and_hole_determinant_is_conjugate():
    """Sec. 2: p[phi] ~ det(M M^dag) > 0.  In the particle-hole basis the hole operator is
    M[-phi, -kappa]; bipartiteness makes det M[-phi,-kappa] = conj det M[phi,kappa], so the
    particle x hole determinant equals det(M M^dag), real and positive."""
    w = TINY
    phi, _ = draw_inputs(w)
    op = _op(w)
    opm = O.HubbardOperator(w.L, w.Nt, w.beta, -w.kappa)
    d1 = np.linalg.det(op.dense_M(phi))
    d2 = np.linalg.det(opm.dense_M(-phi))
    assert abs(d2 - np.conj(d1)) < 1e-12 * abs(d1)
    M = op.dense_M(phi)
    s, ld = np.linalg.slogdet(M @ M.conj().T)
    assert abs(s - 1) < 1e-12 and abs(ld - 2 * np.log(abs(d1))) < 1e-10


# ----------------------------------------------------------------------------- operators
@pytest.mark.parametrize("w", [TINY, SMALL])
def test_adjointness(w):
    """<u, M v> = <M^dag u, v> for the matrix-free operators (P6)."""
    phi, u = draw_inputs(w, seed=1)
    v = draw_complex(w, seed=2)
    op = _op(w)
    lhs = np.vdot(u, op.apply_M(phi, v))
    rhs = np.vdot(op.apply_Mdag(phi, u), v)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_matrix_free_equals_dense_and_expm_route():
    """Matrix-free M, M^dag equal the dense N x N matrix and its conjugate transpose;
    the Krylov-exp route equals the eigh route."""
    w = TINY
    phi, v = draw_inputs(w, seed=4)
    op = _op(w)
    ope = _op(w, mode="expm")
    M = op.dense_M(phi)
    np.testing.assert_allclose(op.apply_M(phi, v).ravel(), M @ v.ravel(), atol=1e-14)
    np.testing.assert_allclose(op.apply_Mdag(phi, v).ravel(), M.conj().T @ v.ravel(), atol=1e-14)
    np.testing.assert_allclose(ope.apply_M(phi, v), op.apply_M(phi, v), atol=1e-13)
    np.testing.assert_allclose(ope.apply_Mdag(phi, v), op.apply_Mdag(phi, v), atol=1e-13)


@pytest.mark.parametrize("L,Nt,beta", [(3, 8, 2.0), (6, 16, 4.0), (12, 8, 1.0)])
def test_free_plane_waves_are_eigenvectors(L, Nt, beta):
    """phi = 0: M acts on (omega_n, k, band) plane waves by 1 - e^{-i omega} e^{delta eps}."""
    op = O.HubbardOperator(L, Nt, beta, mode="expm" if L > 6 else None)
    phi = np.zeros((Nt, 2 * L * L))
    rng = np.random.default_rng(5)
    for _ in range(6):
        n, m1, m2 = rng.integers(Nt), rng.integers(L), rng.integers(L)
        band = rng.choice([-1, 1])
        v, eps, om = CF.plane_wave(L, Nt, n, m1, m2, band)
        lam = CF.free_M_eigenvalue(eps, om, beta / Nt)
        np.testing.assert_allclose(op.apply_M(phi, v[None])[0], lam * v, atol=1e-13)
        np.testing.assert_allclose(op.apply_Mdag(phi, v[None])[0], np.conj(lam) * v, atol=1e-13)


def test_translation_and_time_covariance():
    """Translating phi and chi by a unit cell translates x and the force (P11); rolling
    them by one slice (wrapped chi slice negated) does the same in time (P12)."""
    w = TINY
    L = w.L
    phi, chi = draw_inputs(w)
    op = _op(w)
    x = O.dense_solve(op, phi, chi)
    g = O.force(op, phi, x)

    def shift(a):            # n1 -> n1 + 1 on both sublattices
        s = a.reshape(a.shape[:-1] + (2, L, L))
        return np.roll(s, 1, axis=-2).reshape(a.shape)
    x2 = O.dense_solve(op, shift(phi), shift(chi))
    np.testing.assert_allclose(x2, shift(x), atol=1e-10 * np.abs(x).max())
    np.testing.assert_allclose(O.force(op, shift(phi), x2), shift(g), atol=1e-9 * np.abs(g).max())

    def troll(a, negate):
        r = np.roll(a, 1, axis=-2)
        if negate:
            r[..., 0, :] *= -1
        return r
    x3 = O.dense_solve(op, troll(phi, False), troll(chi, True))
    np.testing.assert_allclose(x3, troll(x, True), atol=1e-10 * np.abs(x).max())
    np.testing.assert_allclose(O.force(op, troll(phi, False), x3), troll(g, False),
                               atol=1e-9 * np.abs(g).max())


# ----------------------------------------------------------------------------- solver
def test_cg_matches_dense_solve():
    w = TINY
    phi, chi = draw_inputs(w)
    op = _op(w)
    x_ref = O.dense_solve(op, phi, chi)
    x, its, res = O.cg_solve(op, phi, chi, tol=1e-12)
    assert res[0] < 1e-11
    M = op.dense_M(phi)
    cond = np.linalg.cond(M @ M.conj().T)
    assert np.linalg.norm(x - x_ref) <= 10 * cond * 1e-12 * np.linalg.norm(x_ref)


@pytest.mark.parametrize("w", [TINY, SMALL])
def test_heat_bath_identity(w):
    """Sec. 2: chi = M rho  =>  M^dag x = rho and S = rho^dag rho."""
    op = _op(w)
    phi = draw_inputs(w)[0]
    rho = draw_complex(w, seed=7)
    chi = op.apply_M(phi, rho)
    if w.N <= 2000:
        x = O.dense_solve(op, phi, chi)
        tol = 1e-9
    else:
        x, _, res = O.cg_solve(op, phi, chi, tol=1e-12)
        tol = 1e-8
    y = op.apply_Mdag(phi, x)
    assert np.linalg.norm(y - rho) <= tol * np.linalg.norm(rho)
    S = O.action(chi, x)
    assert abs(S - np.vdot(rho, rho).real) <= tol * abs(S)


def test_free_plane_wave_solve():
    """phi = 0, plane-wave chi: x = chi / |1 - e^{-i omega} e^{delta eps}|^2 exactly."""
    L, Nt, beta = 6, 16, 4.0
    op = O.HubbardOperator(L, Nt, beta)
    phi = np.zeros((Nt, 2 * L * L))
    v, eps, om = CF.plane_wave(L, Nt, 3, 1, 4, -1)
    lam = CF.free_M_eigenvalue(eps, om, beta / Nt)
    x, _, _ = O.cg_solve(op, phi, v[None], tol=1e-14)
    np.testing.assert_allclose(x[0], v / abs(lam) ** 2, atol=1e-13 * np.abs(v).max() / abs(lam) ** 2)


# ----------------------------------------------------------------------------- force
def test_force_matches_dense_derivative():
    """Matrix-free force equals -x^dag dA x from explicitly assembled dM (1 and 2 RHS)."""
    w = TINY
    phi, chi = draw_inputs(w, nrhs=2)
    op = _op(w)
    x = O.dense_solve(op, phi, chi)
    g = O.force(op, phi, x)
    gd = O.force_dense(op, phi, x)
    assert np.linalg.norm(g - gd) <= 1e-13 * np.linalg.norm(gd)


def _S(op, phi, chi):
    return O.action(chi, O.dense_solve(op, phi, chi))


def test_force_central_finite_differences():
    """dS/dphi against central differences of S (dense solves), eps = 1e-6."""
    w = TINY
    phi, chi = draw_inputs(w)
    op = _op(w)
    g = O.force(op, phi, O.dense_solve(op, phi, chi)).ravel()
    idx = pick_entries(w, 16)
    eps = 1e-6
    gfd = []
    for i in idx:
        pp = phi.copy().ravel(); pp[i] += eps
        pm = phi.copy().ravel(); pm[i] -= eps
        gfd.append((_S(op, pp.reshape(phi.shape), chi) - _S(op, pm.reshape(phi.shape), chi)) / (2 * eps))
    gfd = np.array(gfd)
    assert np.linalg.norm(gfd - g[idx]) <= 1e-6 * np.linalg.norm(g[idx])


def fd_exact_difference(op, phi, chi, i, eps):
    """S(phi + eps e_i) - S(phi - eps e_i) without cancellation.

    M(phi) differs from M with column c = (t, z) removed by the column u(phi) =
    e_c - B_{t+1} e^{i phi_{t,z}} E[:, z] (in slice t+1), so
    A_- - A_+ = u_- u_-^dag - u_+ u_+^dag and
    S_+ - S_- = x_+^dag (A_- - A_+) x_-.
    """
    t, z = divmod(int(i), op.V)
    V = op.V
    tn = (t + 1) % op.Nt

    def col(p):
        u = np.zeros(op.N, dtype=complex)
        u[t * V + z] += 1.0
        u[tn * V:(tn + 1) * V] += -op.B[tn] * np.exp(1j * p) * op.E[:, z]
        return u
    pp = phi.copy().ravel(); pp[i] += eps
    pm = phi.copy().ravel(); pm[i] -= eps
    xp = O.dense_solve(op, pp.reshape(phi.shape), chi).reshape(-1, op.N)
    xm = O.dense_solve(op, pm.reshape(phi.shape), chi).reshape(-1, op.N)
    up, um = col(pp[i]), col(pm[i])
    tot = 0.0
    for a, b in zip(xp, xm):
        tot += (np.vdot(a, um) * np.vdot(um, b) - np.vdot(a, up) * np.vdot(up, b)).real
    return tot


@pytest.mark.slow
def test_force_fd_on_diff_subinstance():
    """18-site torus at Nt = 64, beta = 8, U = 3.8: 64 entries, eps = 1e-6, cancellation-free
    differences; norm-wise error within the conditioning-limited bound."""
    w = DIFF_SUB
    phi, chi = draw_inputs(w)
    op = _op(w)
    x = O.dense_solve(op, phi, chi)
    g = O.force(op, phi, x).ravel()
    gd = O.force_dense(op, phi, x).ravel()
    # |x| ~ cond * |chi| here, so both assemblies cancel large terms
    assert np.linalg.norm(g - gd) <= 1e-10 * np.linalg.norm(gd)
    idx = pick_entries(w, 64)
    eps = 1e-6
    gfd = np.array([fd_exact_difference(op, phi, chi, i, eps) / (2 * eps) for i in idx])
    M = op.dense_M(phi)
    cond = np.linalg.cond(M @ M.conj().T)
    err = np.linalg.norm(gfd - g[idx]) / np.linalg.norm(g[idx])
    # truncation ~ eps^2 * S''' plus roundoff ~ cond * 1e-16 / eps
    assert err < max(1e-8, 1e-16 * cond / eps * 10), (err, cond)


def test_force_fd_exact_difference_tiny():
    w = TINY
    phi, chi = draw_inputs(w)
    op = _op(w)
    g = O.force(op, phi, O.dense_solve(op, phi, chi)).ravel()
    idx = pick_entries(w, 32)
    eps = 1e-5
    gfd = np.array([fd_exact_difference(op, phi, chi, i, eps) / (2 * eps) for i in idx])
    assert np.linalg.norm(gfd - g[idx]) <= 1e-8 * np.linalg.norm(g[idx])


@pytest.mark.parametrize("w", [TINY, SMALL])
def test_force_gauge_sum_rule(w):
    """Slice-uniform gauge transforms G = e^{i theta_t} give M[phi_t + theta_{t+1} - theta_t]
    = G M G^dag, hence sum_x g_{s-1,x} - sum_x g_{s,x} = -2 Im(chi_s^dag x_s) for every s."""
    phi, chi = draw_inputs(w)
    op = _op(w)
    if w.N <= 2000:
        x = O.dense_solve(op, phi, chi)
    else:
        x, _, _ = O.cg_solve(op, phi, chi, tol=1e-13)
    g = O.force(op, phi, x)
    lhs = np.roll(g.sum(axis=1), 1) - g.sum(axis=1)
    rhs = -2 * np.einsum("rtx,rtx->t", np.conj(chi), x).imag
    scale = np.abs(g).sum(axis=1).max()
    np.testing.assert_allclose(lhs, rhs, atol=1e-9 * scale)


def test_degenerate_sizes():
    """L = 1 (all three bonds to one site), Nt = 1 and Nt = 2 stay consistent with the
    closed form and with adjointness."""
    for L, Nt, beta in [(1, 1, 0.5), (1, 2, 1.0), (2, 1, 0.3), (2, 2, 0.7)]:
        op = O.HubbardOperator(L, Nt, beta)
        V = 2 * L * L
        _, ld = np.linalg.slogdet(op.dense_M(np.zeros((Nt, V))))
        assert abs(ld - CF.free_log_det(L, beta).real) < 1e-12
        rng = np.random.default_rng(L * 10 + Nt)
        phi = rng.normal(size=(Nt, V))
        u = rng.normal(size=(1, Nt, V)) + 1j * rng.normal(size=(1, Nt, V))
        v = rng.normal(size=(1, Nt, V)) + 1j * rng.normal(size=(1, Nt, V))
        M = op.dense_M(phi)
        np.testing.assert_allclose(op.apply_M(phi, v).ravel(), M @ v.ravel(), atol=1e-13)
        np.testing.assert_allclose(op.apply_Mdag(phi, u).ravel(), M.conj().T @ u.ravel(), atol=1e-13)


# ----------------------------------------------------------------------------- chemical potential
@pytest.mark.parametrize("mu", [0.3, -0.7])
def test_free_log_det_with_chemical_potential(mu):
    """phi = 0: det M[0, mu] = prod_{k,+-} (1 + e^{beta (mu +- kappa |f(k)|)}) (free fermions
    in the grand-canonical ensemble; Sec. 1 Hamiltonian with mu)."""
    L, Nt, beta = 3, 8, 2.0
    op = O.HubbardOperator(L, Nt, beta, mu=mu)
    _, ld = np.linalg.slogdet(op.dense_M(np.zeros((Nt, 2 * L * L))))
    a = np.abs(CF.f_of_k(L)).ravel()
    ref = np.sum(np.log1p(np.exp(beta * (mu + a)))) + np.sum(np.log1p(np.exp(beta * (mu - a))))
    assert abs(ld - ref) < 1e-11 * abs(ref)


def test_weight_away_from_half_filling_is_not_positive():
    """Sec. 3: det(M[phi,mu] M[phi,-mu]^dag) is real and positive at mu = 0 but complex for
    mu != 0 (the sign problem); at phi = 0 it stays positive."""
    w = TINY
    phi, _ = draw_inputs(w)
    for mu, complex_expected in ((0.0, False), (0.4, True)):
        Mp = O.HubbardOperator(w.L, w.Nt, w.beta, mu=mu).dense_M(phi)
        Mm = O.HubbardOperator(w.L, w.Nt, w.beta, mu=-mu).dense_M(phi)
        sign, _ = np.linalg.slogdet(Mp @ Mm.conj().T)
        assert (abs(np.angle(sign)) > 1e-6) == complex_expected, (mu, sign)
        Mp0 = O.HubbardOperator(w.L, w.Nt, w.beta, mu=mu).dense_M(np.zeros_like(phi))
        Mm0 = O.HubbardOperator(w.L, w.Nt, w.beta, mu=-mu).dense_M(np.zeros_like(phi))
        s0, _ = np.linalg.slogdet(Mp0 @ Mm0.conj().T)
        assert abs(s0 - 1) < 1e-10


def test_chemical_potential_routes_agree():
    """e^{delta mu} on the Krylov-exp route equals the dense route; adjointness holds."""
    w = TINY
    phi, v = draw_inputs(w, seed=8)
    u = draw_complex(w, seed=9)
    op = O.HubbardOperator(w.L, w.Nt, w.beta, mu=0.5)
    ope = O.HubbardOperator(w.L, w.Nt, w.beta, mu=0.5, mode="expm")
    np.testing.assert_allclose(ope.apply_M(phi, v), op.apply_M(phi, v), atol=1e-13)
    np.testing.assert_allclose(op.dense_M(phi) @ v.ravel(), op.apply_M(phi, v).ravel(), atol=1e-13)
    a = np.vdot(u, op.apply_M(phi, v))
    b = np.vdot(op.apply_Mdag(phi, u), v)
    assert abs(a - b) < 1e-12 * abs(a)


# ----------------------------------------------------------------------------- Sec. 3 weight
def test_oracle_log_det_routes():
    """The transfer-product log det equals the dense slogdet of M (any field, mu = 0 and mu != 0)
    and the free closed form with a chemical potential; the sign phase is zero at mu = 0 and
    at phi = 0, nonzero on a random field at mu != 0 (Sec. 3: the sign problem)."""
    w = TINY
    phi, _ = draw_inputs(w)
    for mu in (0.0, 0.4, -0.9):
        op = O.HubbardOperator(w.L, w.Nt, w.beta, mu=mu)
        s, ld = np.linalg.slogdet(op.dense_M(phi))
        l2, a2 = O.log_det(op, phi)
        assert abs(ld - l2) < 1e-11 * abs(ld) and abs(np.exp(1j * a2) - s) < 1e-11
        l0, a0 = O.log_det(op, np.zeros_like(phi))
        a = np.abs(CF.f_of_k(w.L)).ravel()
        ref = np.sum(np.log1p(np.exp(w.beta * (mu + a)))) + np.sum(np.log1p(np.exp(w.beta * (mu - a))))
        assert abs(l0 - ref) < 1e-11 * abs(ref) and abs(a0) < 1e-12
    opp = O.HubbardOperator(w.L, w.Nt, w.beta, mu=0.4)
    opm = O.HubbardOperator(w.L, w.Nt, w.beta, mu=-0.4)
    op0 = O.HubbardOperator(w.L, w.Nt, w.beta)
    assert abs(O.sign_phase(op0, op0, phi)) == 0.0
    assert abs(O.sign_phase(opp, opm, np.zeros_like(phi))) < 1e-12
    th = O.sign_phase(opp, opm, phi)
    Mp, Mm = opp.dense_M(phi), opm.dense_M(phi)
    s, _ = np.linalg.slogdet(Mp @ Mm.conj().T)
    assert abs(np.exp(1j * th) - s) < 1e-10 and abs(th) > 1e-6


def test_reweighting_identity():
    """<O>_p = <O e^{i theta}>_|p| / <e^{i theta}>_|p|: for samples drawn with weights |p_i| of a
    finite set, the ratio equals the exact sum over the set with the complex weights p_i."""
    rng = np.random.default_rng(4)
    n = 6
    p = rng.uniform(0.1, 1.0, n) * np.exp(1j * rng.uniform(-2.5, 2.5, n))
    obs = rng.normal(size=n)
    exact = np.sum(obs * p) / np.sum(p)
    draws = rng.choice(n, size=400000, p=np.abs(p) / np.abs(p).sum())
    est = O.reweight(obs[draws], np.angle(p)[draws])
    assert abs(est - exact) < 0.02 * abs(exact)
