"""GPU parity of the linear form of the fermion matrix (eq. "ferm_op" as printed): the
stencil operators, the solver on them, the force and an HMC trajectory, through the C ABI,
against the oracle's LinearHubbardOperator."""
import numpy as np
import pytest

import oracle as O
from oracle import hmc as OH
from workloads import TINY, SMALL, PREC, STRESS, Lattice, draw_inputs, draw_complex, draw_weak_field, \
    draw_hmc_randoms, pick_entries
from gpu_common import to_dev, to_np, assert_close_elementwise
import closed_forms as CF

pytestmark = pytest.mark.gpu

RTOL64 = 1e-14     # five terms per entry, each rounded once or twice in FP64
RTOL32 = 1e-6      # the same in FP32 (phase from the FP32 angle)


def _hub(w, nrhs=1):
    from paper_2210_06874_amd import Hubbard
    return Hubbard(w.L, w.Nt, w.beta, w.kappa, nrhs_max=nrhs, form="linear")


def _op(w):
    return O.LinearHubbardOperator(w.L, w.Nt, w.beta, w.kappa)


EDGE = [
    Lattice("L1_Nt1", 1, 1, 0.5, 3.0), Lattice("L1_Nt2", 1, 2, 1.0, 3.0),
    Lattice("L2_Nt2", 2, 2, 0.7, 3.0), Lattice("L5_Nt3", 5, 3, 1.5, 3.0),
    Lattice("L19_Nt4", 19, 4, 2.0, 3.0),       # prime above the DFT radices: fine for a stencil
    Lattice("L23_Nt7", 23, 7, 2.0, 3.0),       # V = 1058: two chunks per slice
    Lattice("L6_Nt9", 6, 9, 3.0, 3.0),
]


@pytest.mark.parametrize("w", [TINY, SMALL] + EDGE, ids=lambda w: w.name)
def test_apply_fp64_matches_oracle(w):
    print(f"[case] linear apply fp64 {w.name}", flush=True)
    phi, v = draw_inputs(w, seed=61, nrhs=2)
    hub = _hub(w, nrhs=2)
    assert hub.path == "fused" and hub.lds_bytes == 0
    op = _op(w)
    assert_close_elementwise(to_np(hub.apply_M(to_dev(phi), to_dev(v))), op.apply_M(phi, v), RTOL64, "M")
    assert_close_elementwise(to_np(hub.apply_Mdag(to_dev(phi), to_dev(v))), op.apply_Mdag(phi, v), RTOL64, "Mdag")


@pytest.mark.parametrize("w", [TINY, SMALL, EDGE[4], EDGE[5]], ids=lambda w: w.name)
def test_apply_fp32_matches_oracle(w):
    print(f"[case] linear apply fp32 {w.name}", flush=True)
    phi, v = draw_inputs(w, seed=62)
    phi32, v64 = phi.astype(np.float32), v.astype(np.complex64)
    hub = _hub(w)
    op = _op(w)
    p, x = phi32.astype(np.float64), v64.astype(np.complex128)
    assert_close_elementwise(to_np(hub.apply_M_c64(to_dev(phi32), to_dev(v64))), op.apply_M(p, x), RTOL32, "M32")
    assert_close_elementwise(to_np(hub.apply_Mdag_c64(to_dev(phi32), to_dev(v64))), op.apply_Mdag(p, x), RTOL32,
                             "Mdag32")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_precision_workload(prec):
    """L = 51, Nt = 128, every entry (the stencil oracle is cheap at this size)."""
    w = PREC
    print(f"[case] linear apply {prec} {w.name}", flush=True)
    phi, v = draw_inputs(w, seed=63)
    hub = _hub(w)
    op = _op(w)
    if prec == "fp64":
        got_M, got_D = hub.apply_M(to_dev(phi), to_dev(v)), hub.apply_Mdag(to_dev(phi), to_dev(v))
        tol = RTOL64
    else:
        phi, v = phi.astype(np.float32), v.astype(np.complex64)
        got_M, got_D = hub.apply_M_c64(to_dev(phi), to_dev(v)), hub.apply_Mdag_c64(to_dev(phi), to_dev(v))
        phi, v = phi.astype(np.float64), v.astype(np.complex128)
        tol = RTOL32
    assert_close_elementwise(to_np(got_M), op.apply_M(phi, v), tol, "M")
    assert_close_elementwise(to_np(got_D), op.apply_Mdag(phi, v), tol, "Mdag")


def test_stress_workload_sampled_rows():
    """L = 102, Nt = 192, four right-hand sides: sampled entries against the oracle."""
    w = STRESS
    print(f"[case] linear apply {w.name}", flush=True)
    phi, v = draw_inputs(w, seed=64, nrhs=w.nrhs)
    hub = _hub(w, nrhs=w.nrhs)
    op = _op(w)
    got = to_np(hub.apply_M(to_dev(phi), to_dev(v)))
    ref = op.apply_M(phi, v)
    idx = pick_entries(w, 4000)
    assert_close_elementwise(got.reshape(w.nrhs, -1)[:, idx], ref.reshape(w.nrhs, -1)[:, idx], RTOL64, "M")


def test_adjointness_and_plane_wave_at_full_size():
    """<u, M v> = <M^dag u, v> in FP64 at L = 51, Nt = 128; at phi = 0 a free plane wave
    is an eigenvector of the 2 x 2 momentum block."""
    w = PREC
    phi, v = draw_inputs(w, seed=65)
    u = draw_complex(w, seed=66)
    hub = _hub(w)
    Mv = to_np(hub.apply_M(to_dev(phi), to_dev(v)))
    Du = to_np(hub.apply_Mdag(to_dev(phi), to_dev(u)))
    a, b = np.vdot(u, Mv), np.vdot(Du, v)
    assert abs(a - b) <= 1e-12 * abs(a)
    L, Nt = w.L, w.Nt
    dk = w.delta * w.kappa
    n, m1, m2 = 5, 7, 30
    om = (2 * n + 1) * np.pi / Nt
    f = 1 + np.exp(-2j * np.pi * m1 / L) + np.exp(-2j * np.pi * m2 / L)
    blk = np.array([[np.exp(1j * om) - 1, -dk * f], [-dk * np.conj(f), 1 - np.exp(-1j * om)]])
    lam, vec = np.linalg.eig(blk)
    n1, n2 = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    ph = np.exp(2j * np.pi * ((m1 * n1 + m2 * n2) % L) / L).ravel()
    tt = np.exp(1j * np.pi * ((2 * n + 1) * np.arange(Nt) % (2 * Nt)) / Nt)
    x = tt[:, None] * np.concatenate([vec[0, 0] * ph, vec[1, 0] * ph])[None, :]
    got = to_np(hub.apply_M(to_dev(np.zeros((Nt, w.V))), to_dev(x)))
    assert np.abs(got - lam[0] * x).max() <= 1e-13


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cg_tiny_against_dense_solve(prec):
    w = TINY
    print(f"[case] linear cg {prec} {w.name}", flush=True)
    phi, chi = draw_inputs(w, seed=67, nrhs=2)
    op = _op(w)
    ref = O.dense_solve_op(op, phi, chi)
    hub = _hub(w, nrhs=2)
    res = hub.cg_solve(to_dev(phi), to_dev(chi), tol=1e-12, prec=prec)
    assert res.converged and max(res.true_rel_res) <= 1e-12
    x = to_np(res.x)
    A = op.dense_M(phi)
    A = A @ A.conj().T
    cond = np.linalg.cond(A)
    assert np.linalg.norm(x - ref) <= 2 * cond * 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("w", [SMALL, PREC], ids=lambda w: w.name)
def test_cg_weak_field_true_residual(w, prec):
    """The oracle recomputes ||chi - M M^dag x|| / ||chi|| from the returned x."""
    print(f"[case] linear cg {prec} {w.name}", flush=True)
    phi, chi = draw_weak_field(w, seed=68)
    hub = _hub(w)
    res = hub.cg_solve(to_dev(phi), to_dev(chi), tol=1e-10, prec=prec, max_iter=20000)
    assert res.converged
    op = _op(w)
    x = to_np(res.x)
    rr = np.linalg.norm(chi - op.apply_A(phi, x)) / np.linalg.norm(chi)
    assert rr <= 1.01e-10, rr
    assert abs(rr - res.true_rel_res[0]) <= 1e-3 * rr + 1e-15


def test_cg_small_matches_oracle_cg():
    w = SMALL
    phi, chi = draw_weak_field(w, seed=69)
    op = _op(w)
    xo, _, _ = O.cg_solve(op, phi, chi, tol=1e-12)
    hub = _hub(w)
    res = hub.cg_solve(to_dev(phi), to_dev(chi), tol=1e-12, prec="mixed")
    assert res.converged
    assert np.linalg.norm(to_np(res.x) - xo) <= 1e-8 * np.linalg.norm(xo)


def test_cg_batched_equals_single():
    w = SMALL
    phi, chi = draw_weak_field(w, seed=70)
    chi2 = np.stack([chi[0], 0.5 * chi[0] + draw_complex(w, seed=71)[0], np.zeros_like(chi[0])])
    hub = _hub(w, nrhs=3)
    batched = hub.cg_solve(to_dev(phi), to_dev(chi2), tol=1e-10, prec="mixed")
    assert batched.converged
    assert np.all(to_np(batched.x)[2] == 0)
    for r in range(2):
        single = hub.cg_solve(to_dev(phi), to_dev(chi2[r]), tol=1e-10, prec="mixed")
        assert single.converged
        ref = to_np(single.x)
        assert np.linalg.norm(to_np(batched.x)[r] - ref) <= 1e-8 * np.linalg.norm(ref)


@pytest.mark.parametrize("w", [TINY, SMALL, EDGE[0], EDGE[2], EDGE[4], PREC], ids=lambda w: w.name)
def test_force_kernel_matches_oracle(w):
    print(f"[case] linear force {w.name}", flush=True)
    nrhs = 1 if w is PREC else 2
    phi, x = draw_inputs(w, seed=72, nrhs=nrhs)
    hub = _hub(w, nrhs=nrhs)
    got = to_np(hub.force(to_dev(phi), to_dev(x)))
    assert_close_elementwise(got, O.force_linear(_op(w), phi, x), 1e-13, "force")


def test_force_end_to_end_tiny_dense():
    w = TINY
    phi, chi = draw_inputs(w, seed=73)
    op = _op(w)
    g_ref = O.force_dense_linear(op, phi, O.dense_solve_op(op, phi, chi))
    hub = _hub(w)
    res = hub.cg_solve(to_dev(phi), to_dev(chi), tol=1e-13, max_iter=20000)
    g = to_np(hub.force(to_dev(phi), res.x))
    assert np.linalg.norm(g - g_ref) <= 1e-8 * np.linalg.norm(g_ref)


@pytest.mark.parametrize("integrator", ["leapfrog", "omelyan"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_trajectory_matches_oracle(prec, integrator):
    from paper_2210_06874_amd import hmc
    w = TINY
    print(f"[case] linear hmc trajectory {prec} {integrator} {w.name}", flush=True)
    phi0 = draw_weak_field(w)[0]
    op = _op(w)
    hub = _hub(w)
    for pi, rho, u in draw_hmc_randoms(w, 2, seed=74):
        _, _, dH_ref, acc_ref, out_ref = OH.trajectory(op, w.U, phi0, pi, rho, u, n_md=8, eps=0.05,
                                                       integrator=integrator)
        P = to_dev(phi0)
        tr = hmc.trajectory(hub, P, w.U, to_dev(pi), to_dev(rho), u, n_md=8, eps=0.05, tol=1e-12, prec=prec,
                            integrator=integrator)
        assert abs(tr.dH - dH_ref) <= 1e-7 * max(1.0, abs(dH_ref)), (tr.dH, dH_ref)
        assert tr.accepted == acc_ref
        np.testing.assert_allclose(to_np(P), out_ref, atol=1e-8)
        phi0 = out_ref


def test_linear_form_rejects_mu():
    from paper_2210_06874_amd import Hubbard, HubError
    with pytest.raises(HubError):
        Hubbard(3, 8, 2.0, 1.0, mu=0.3, form="linear")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cg_free_plane_wave_at_full_size(prec):
    """phi = 0: a plane wave carrying an eigenvector of the momentum block's B B^dag is an
    eigenvector of M M^dag, so x = chi / sigma^2 (L = 51, N_t = 128)."""
    w = PREC
    L, Nt = w.L, w.Nt
    dk = w.delta * w.kappa
    n, m1, m2 = 3, 5, 40
    om = (2 * n + 1) * np.pi / Nt
    f = 1 + np.exp(-2j * np.pi * m1 / L) + np.exp(-2j * np.pi * m2 / L)
    blk = np.array([[np.exp(1j * om) - 1, -dk * f], [-dk * np.conj(f), 1 - np.exp(-1j * om)]])
    s2, vec = np.linalg.eigh(blk @ blk.conj().T)
    n1, n2 = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    ph = np.exp(2j * np.pi * ((m1 * n1 + m2 * n2) % L) / L).ravel()
    tt = np.exp(1j * np.pi * ((2 * n + 1) * np.arange(Nt) % (2 * Nt)) / Nt)
    hub = _hub(w)
    phi = np.zeros((Nt, w.V))
    for j in range(2):
        chi = tt[:, None] * np.concatenate([vec[0, j] * ph, vec[1, j] * ph])[None, :]
        res = hub.cg_solve(to_dev(phi), to_dev(chi), tol=1e-10, prec=prec)
        assert res.converged
        err = np.linalg.norm(to_np(res.x) - chi / s2[j]) / np.linalg.norm(chi / s2[j])
        assert err <= 2 * _free_cond_linear(w) * 1e-10, (j, err)


def _free_cond_linear(w):
    """cond(M M^dag) of the linear form at phi = 0: extreme singular values of the 2 x 2
    momentum blocks over all Matsubara frequencies and momenta."""
    om = (2 * np.arange(w.Nt) + 1) * np.pi / w.Nt
    dk = w.delta * w.kappa
    g = (dk * np.abs(CF.f_of_k(w.L)).ravel())[None, :]
    a = (np.exp(1j * om) - 1)[:, None] * np.ones_like(g)
    d = (1 - np.exp(-1j * om))[:, None] * np.ones_like(g)
    # B B^dag for B = [[a, -g u], [-g conj(u), d]] with |u| = 1 has trace and determinant:
    tr = np.abs(a) ** 2 + np.abs(d) ** 2 + 2 * g ** 2
    det = np.abs(a * d - g ** 2) ** 2
    disc = np.sqrt(np.maximum(tr ** 2 - 4 * det, 0))
    return ((tr + disc) / 2).max() / ((tr - disc) / 2).min()


def test_apply_maximum_lattice():
    """L = 1024, N_t = 2 (the largest torus the ABI accepts), every entry of M and M^dag."""
    w = Lattice("L1024_Nt2", 1024, 2, 0.5, 3.0)
    print(f"[case] linear apply {w.name}", flush=True)
    phi, v = draw_inputs(w, seed=75)
    hub = _hub(w)
    op = _op(w)
    assert_close_elementwise(to_np(hub.apply_M(to_dev(phi), to_dev(v))), op.apply_M(phi, v), RTOL64, "M")
    assert_close_elementwise(to_np(hub.apply_Mdag(to_dev(phi), to_dev(v))), op.apply_Mdag(phi, v), RTOL64, "Mdag")


@pytest.mark.parametrize("L,Nt,nrhs", [(51, 1, 1), (51, 3, 4), (51, 255, 1), (51, 1024, 1), (102, 5, 3), (102, 1, 2)])
def test_stencil_chunking_at_odd_shapes(L, Nt, nrhs):
    """The chunk count per slice depends on N_t and nrhs (at least 256 workgroups, at most
    1,024 reduction slots): M, M^dag, FP32 M and the force at shapes that give one chunk, many
    chunks and a single slice, against the oracle."""
    from paper_2210_06874_amd import Hubbard
    print(f"[case] stencil chunking L={L} Nt={Nt} nrhs={nrhs}", flush=True)
    w = Lattice(f"L{L}_Nt{Nt}", L, Nt, 0.0625 * Nt, 3.9, nrhs=nrhs)
    phi, v = draw_inputs(w, seed=L + 3 * Nt, nrhs=nrhs)
    op = _op(w)
    hub = Hubbard(L, Nt, w.beta, w.kappa, nrhs_max=nrhs, form="linear")
    P, V = to_dev(phi), to_dev(v)
    assert_close_elementwise(to_np(hub.apply_M(P, V)), op.apply_M(phi, v), 1e-13, "M")
    assert_close_elementwise(to_np(hub.apply_Mdag(P, V)), op.apply_Mdag(phi, v), 1e-13, "Mdag")
    p32, v32 = phi.astype(np.float32), v.astype(np.complex64)
    assert_close_elementwise(to_np(hub.apply_M_c64(to_dev(p32), to_dev(v32))),
                             op.apply_M(p32.astype(np.float64), v32.astype(np.complex128)), 2e-6, "M32")
    assert_close_elementwise(to_np(hub.force(P, V)), O.force_linear(op, phi, v), 1e-12, "force")
