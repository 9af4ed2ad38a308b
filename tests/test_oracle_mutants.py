"""Planted mistakes in the CPU oracle must be caught by the pins.

Each mutant patches one plausible error into the oracle (a wrong sign, a dropped
term, a wrong index or a conjugation slip) and the test asserts that at least one
of the independent checks below rejects it, while the unmodified oracle passes all
of them.  Mistakes are planted only in the oracle, on the CPU.
"""
import contextlib
import math

import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

import oracle as O
import oracle.hubbard as OH
from workloads import TINY, draw_inputs, draw_complex, pick_entries
import closed_forms as CF


def _op():
    w = TINY
    return O.HubbardOperator(w.L, w.Nt, w.beta, w.kappa)


def check_free_logdet():
    w = TINY
    op = _op()
    _, ld = np.linalg.slogdet(op.dense_M(np.zeros((w.Nt, w.V))))
    return abs(ld - CF.free_log_det(w.L, w.beta).real) < 1e-10


def check_plane_wave():
    w = TINY
    op = _op()
    v, eps, om = CF.plane_wave(w.L, w.Nt, 2, 1, 2, 1)
    lam = CF.free_M_eigenvalue(eps, om, w.delta)
    out = op.apply_M(np.zeros((w.Nt, w.V)), v[None])[0]
    return np.abs(out - lam * v).max() < 1e-12


def check_adjoint():
    w = TINY
    phi, u = draw_inputs(w, seed=1)
    v = draw_complex(w, seed=2)
    op = _op()
    a = np.vdot(u, op.apply_M(phi, v))
    b = np.vdot(op.apply_Mdag(phi, u), v)
    return abs(a - b) < 1e-12 * abs(a)


def check_dense_vs_free():
    w = TINY
    phi, v = draw_inputs(w, seed=3)
    op = _op()
    return np.abs(op.dense_M(phi) @ v.ravel() - op.apply_M(phi, v).ravel()).max() < 1e-12


def check_uniform_phase():
    w = TINY
    c = np.linspace(-0.4, 0.9, w.Nt)
    op = _op()
    det = np.linalg.det(op.dense_M(np.repeat(c[:, None], w.V, axis=1)))
    ref = np.exp(CF.free_log_det(w.L, w.beta, total_phase=c.sum()))
    return abs(det - ref) < 1e-10 * abs(ref)


def check_geometry():
    K = O.hopping_matrix(3)
    lam = np.sort(np.linalg.eigvalsh(K))
    a = np.abs(CF.f_of_k(3)).ravel()
    ok = np.allclose(lam, np.sort(np.concatenate([a, -a])), atol=1e-12)
    # brute-force neighbour check on real-space coordinates (see test_oracle_pins)
    a1 = np.array([1.5, math.sqrt(3) / 2])
    a2 = np.array([1.5, -math.sqrt(3) / 2])
    for an, bn in O.honeycomb_bonds(3):
        n1, n2 = divmod(an, 3)
        m1, m2 = divmod(bn - 9, 3)
        pa = n1 * a1 + n2 * a2
        pb = m1 * a1 + m2 * a2 + np.array([1.0, 0.0])
        d = min(np.linalg.norm(pa - pb + i * 3 * a1 + j * 3 * a2) for i in (-1, 0, 1) for j in (-1, 0, 1))
        ok &= abs(d - 1) < 1e-9
    return bool(ok)


def check_solver():
    w = TINY
    phi, chi = draw_inputs(w)
    op = _op()
    M = op.dense_M(phi)
    A = M @ M.conj().T
    x, _, _ = O.cg_solve(op, phi, chi, tol=1e-12)
    return np.linalg.norm(A @ x.ravel() - chi.ravel()) < 1e-9 * np.linalg.norm(chi)


def check_force_fd():
    w = TINY
    phi, chi = draw_inputs(w)
    op = _op()

    def S(p):
        M = op.dense_M(p)
        x = np.linalg.solve(M @ M.conj().T, chi.ravel())
        return np.vdot(chi.ravel(), x).real
    M = op.dense_M(phi)
    x = np.linalg.solve(M @ M.conj().T, chi.ravel()).reshape(chi.shape)
    g = O.force(op, phi, x).ravel()
    eps = 1e-6
    idx = pick_entries(w, 8)
    fd = []
    for i in idx:
        pp = phi.ravel().copy(); pp[i] += eps
        pm = phi.ravel().copy(); pm[i] -= eps
        fd.append((S(pp.reshape(phi.shape)) - S(pm.reshape(phi.shape))) / (2 * eps))
    fd = np.array(fd)
    return np.linalg.norm(fd - g[idx]) < 1e-5 * np.linalg.norm(g[idx])


CHECKS = [check_free_logdet, check_plane_wave, check_adjoint, check_dense_vs_free,
          check_uniform_phase, check_geometry, check_solver, check_force_fd]


# ----------------------------------------------------------------------------- mutants
@contextlib.contextmanager
def patched(obj, name, new):
    old = getattr(obj, name)
    setattr(obj, name, new)
    try:
        yield
    finally:
        setattr(obj, name, old)


def periodic_signs(Nt):
    return np.ones(Nt)


def wrap_sign_on_last(Nt):
    B = np.ones(Nt)
    B[-1] = -1.0
    return B


def bonds_wrong_direction(L):
    out = []
    for n1 in range(L):
        for n2 in range(L):
            a = O.site_index(L, 0, n1, n2)
            for d1, d2 in ((0, 0), (1, 0), (0, -1)):
                out.append((a, O.site_index(L, 1, n1 + d1, n2 + d2)))
    return out


def apply_M_no_identity(self, phi, v):
    vv, shp = self._shape(v)
    src = np.roll(np.exp(1j * phi)[None] * vv, 1, axis=1)
    return (-self.B[None, :, None] * self.apply_E(src)).reshape(shp)


def apply_M_conj_phase(self, phi, v):
    vv, shp = self._shape(v)
    src = np.roll(np.exp(-1j * phi)[None] * vv, 1, axis=1)
    return (vv - self.B[None, :, None] * self.apply_E(src)).reshape(shp)


def apply_M_phase_on_target(self, phi, v):
    vv, shp = self._shape(v)
    src = np.roll(vv, 1, axis=1)
    return (vv - self.B[None, :, None] * np.exp(1j * phi)[None] * self.apply_E(src)).reshape(shp)


def apply_Mdag_wrong_sign_slot(self, phi, v):
    vv, shp = self._shape(v)
    hop = np.roll(self.apply_E(vv), -1, axis=1)
    return (vv - self.B[None, :, None] * np.exp(-1j * phi)[None] * hop).reshape(shp)


_ORIG_FORCE = OH.force


def force_sign_flipped(op, phi, x):
    return -_ORIG_FORCE(op, phi, x)


def force_no_factor_two(op, phi, x):
    return 0.5 * _ORIG_FORCE(op, phi, x)


def force_wrong_slice(op, phi, x):
    xx = np.asarray(x, dtype=np.complex128).reshape(-1, op.Nt, op.V)
    g = np.zeros((op.Nt, op.V))
    Bn = np.roll(op.B, -1)[:, None]
    for xr in xx:
        y = op.apply_Mdag(phi, xr)
        w = op.apply_E(xr)                          # E x_t instead of E x_{t+1}
        g += 2.0 * (Bn * 1j * np.exp(1j * phi) * y * np.conj(w)).real
    return g


def cg_no_conj(op, phi, chi, tol=1e-12, max_iter=100000, x0=None):
    chi = np.asarray(chi).reshape(-1, op.Nt, op.V)
    out = []
    for c in chi:
        x = np.zeros_like(c); r = c.copy(); p = r.copy()
        rr = np.sum(r * r).real
        for _ in range(400):
            q = op.apply_A(phi, p)
            a = rr / np.sum(p * q).real
            x = x + a * p; r = r - a * q
            rn = np.sum(r * r).real
            p = r + rn / rr * p; rr = rn
        out.append(x)
    return np.stack(out), None, None


MUTANTS = {
    "periodic_time": lambda: patched(OH, "antiperiodic_signs", periodic_signs),
    "wrap_sign_wrong_block": lambda: patched(OH, "antiperiodic_signs", wrap_sign_on_last),
    "bond_direction": lambda: patched(OH, "honeycomb_bonds", bonds_wrong_direction),
    "M_drops_identity": lambda: patched(OH.HubbardOperator, "apply_M", apply_M_no_identity),
    "M_conjugated_phase": lambda: patched(OH.HubbardOperator, "apply_M", apply_M_conj_phase),
    "M_phase_on_target": lambda: patched(OH.HubbardOperator, "apply_M", apply_M_phase_on_target),
    "Mdag_sign_index": lambda: patched(OH.HubbardOperator, "apply_Mdag", apply_Mdag_wrong_sign_slot),
    "force_sign": lambda: patched(OH, "force", force_sign_flipped),
    "force_factor": lambda: patched(OH, "force", force_no_factor_two),
    "force_wrong_slice": lambda: patched(OH, "force", force_wrong_slice),
    "cg_missing_conjugate": lambda: patched(OH, "cg_solve", cg_no_conj),
}


def _run_checks():
    res = {}
    for c in CHECKS:
        try:
            res[c.__name__] = bool(c())
        except Exception:
            res[c.__name__] = False
    return res


def test_unmutated_oracle_passes_every_check():
    res = _run_checks()
    assert all(res.values()), res


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    # the oracle package re-exports names; patch both module and package views
    with MUTANTS[name]():
        for attr in ("antiperiodic_signs", "honeycomb_bonds", "force", "cg_solve"):
            monkeypatch.setattr(O, attr, getattr(OH, attr))
        res = _run_checks()
    assert not all(res.values()), f"mutant {name} passed every check: {res}"


# ----------------------------------------------------------------------------- linear form
# Mistakes in the linear form of eq. "ferm_op", planted CONSISTENTLY: the mutated operator's
# dense matrix, matrix-free M and M^dag all agree with each other (so adjointness and
# matrix-free = dense cannot see them); only the fixed facts at phi != 0 can.
from test_oracle_linear import check_uniform_field_momentum_blocks, check_single_site_phase_determinant

_LIN = OH.LinearHubbardOperator


def _lin_mutant(edit):
    """A linear-form operator whose dense matrix is the oracle's with `edit` applied, and whose
    M and M^dag are that matrix and its adjoint."""
    class Mutant(_LIN):
        def dense_M(self, phi):
            M = _LIN.dense_M(self, phi)
            edit(self, np.asarray(phi), M)
            return M

        def apply_M(self, phi, v):
            vv, shp = self._shape(v)
            return (vv.reshape(-1, self.N) @ self.dense_M(phi).T).reshape(shp)

        def apply_Mdag(self, phi, v):
            vv, shp = self._shape(v)
            return (vv.reshape(-1, self.N) @ self.dense_M(phi).conj()).reshape(shp)
    return Mutant


def _b_hop_entries(op):
    for t in range(op.Nt):
        for x in range(op.nA, op.V):
            yield t, x, t * op.V + x, ((t - 1) % op.Nt) * op.V + x


def edit_b_phase_sign(op, phi, M):                  # e^{+i phi} on the B-site hop
    for t, x, r, c in _b_hop_entries(op):
        Bt = -1.0 if t == 0 else 1.0
        M[r, c] = -Bt * np.exp(1j * phi[t, x])


def edit_b_phase_previous_slice(op, phi, M):        # the B hop's phase taken from slice t-1
    for t, x, r, c in _b_hop_entries(op):
        Bt = -1.0 if t == 0 else 1.0
        M[r, c] = -Bt * np.exp(-1j * phi[(t - 1) % op.Nt, x])


def edit_a_wrap_sign(op, phi, M):                   # A's forward hop with B_t instead of B_{t+1}
    for t in range(op.Nt):
        tn = (t + 1) % op.Nt
        for x in range(op.nA):
            M[t * op.V + x, tn * op.V + x] = -1.0 if t == 0 else 1.0


def edit_a_phase_conjugated(op, phi, M):            # e^{-i phi} on the A-site diagonal
    for t in range(op.Nt):
        for x in range(op.nA):
            M[t * op.V + x, t * op.V + x] = -np.exp(-1j * phi[t, x])


def edit_a_phase_next_slice(op, phi, M):            # the A diagonal's phase taken from slice t+1
    for t in range(op.Nt):
        for x in range(op.nA):
            M[t * op.V + x, t * op.V + x] = -np.exp(1j * phi[(t + 1) % op.Nt, x])


def edit_dropped_hopping(op, phi, M):               # delta*kappa dropped
    K = op.K.toarray()
    for t in range(op.Nt):
        M[t * op.V:(t + 1) * op.V, t * op.V:(t + 1) * op.V] += op.dk * K


LIN_MUTANTS = {
    "lin_B_phase_sign": edit_b_phase_sign,
    "lin_B_phase_previous_slice": edit_b_phase_previous_slice,
    "lin_A_wrap_sign": edit_a_wrap_sign,
    "lin_A_phase_conjugated": edit_a_phase_conjugated,
    "lin_A_phase_next_slice": edit_a_phase_next_slice,
    "lin_dropped_hopping": edit_dropped_hopping,
}


def _lin_fixed_facts(cls):
    return [check_uniform_field_momentum_blocks(cls), check_single_site_phase_determinant(cls)]


def test_linear_mutants_are_self_consistent_and_the_unmutated_form_passes():
    """Every mutant keeps M^dag the adjoint of M (so only the fixed facts can catch it), and
    the oracle's own linear form passes both fixed facts."""
    assert all(_lin_fixed_facts(_LIN))
    w = TINY
    phi, u = draw_inputs(w, seed=1)
    v = draw_complex(w, seed=2)
    for edit in LIN_MUTANTS.values():
        op = _lin_mutant(edit)(w.L, w.Nt, w.beta, w.kappa)
        a = np.vdot(u, op.apply_M(phi, v))
        b = np.vdot(op.apply_Mdag(phi, u), v)
        assert abs(a - b) < 1e-12 * abs(a)


@pytest.mark.parametrize("name", sorted(LIN_MUTANTS))
def test_linear_mutant_is_caught_by_a_fixed_fact(name):
    assert not all(_lin_fixed_facts(_lin_mutant(LIN_MUTANTS[name])))


# force mistakes of the linear form, caught by finite differences of the pinned operator
_ORIG_FORCE_LIN = OH.force_linear


def force_linear_sign(op, phi, x):
    return -_ORIG_FORCE_LIN(op, phi, x)


def force_linear_b_same_slice(op, phi, x):
    """B sites paired with y_t instead of y_{t-1}."""
    xx = np.asarray(x, dtype=np.complex128).reshape(-1, op.Nt, op.V)
    g = _ORIG_FORCE_LIN(op, phi, x)
    Bs = slice(op.nA, op.V)
    g[:, Bs] = 0.0
    for xr in xx:
        y = op.apply_Mdag(phi, xr)
        g[:, Bs] += 2.0 * op.B[:, None] * (np.exp(-1j * phi[:, Bs]) * np.conj(xr[:, Bs]) * y[:, Bs]).imag
    return g


def check_linear_force_fd():
    w = TINY
    phi, chi = draw_inputs(w)
    op = O.LinearHubbardOperator(w.L, w.Nt, w.beta, w.kappa)
    x = O.dense_solve_op(op, phi, chi)
    g = OH.force_linear(op, phi, x).ravel()
    eps = 1e-6
    idx = pick_entries(w, 12)
    fd = []
    for i in idx:
        pp = phi.ravel().copy(); pp[i] += eps
        pm = phi.ravel().copy(); pm[i] -= eps
        sp_ = O.action(chi, O.dense_solve_op(op, pp.reshape(phi.shape), chi))
        sm_ = O.action(chi, O.dense_solve_op(op, pm.reshape(phi.shape), chi))
        fd.append((sp_ - sm_) / (2 * eps))
    return np.linalg.norm(np.array(fd) - g[idx]) <= 1e-6 * np.linalg.norm(g[idx])


@pytest.mark.parametrize("mut", [force_linear_sign, force_linear_b_same_slice], ids=lambda f: f.__name__)
def test_linear_force_mutant_is_caught(mut):
    assert check_linear_force_fd()
    with patched(OH, "force_linear", mut):
        assert not check_linear_force_fd()
