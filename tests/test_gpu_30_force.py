"""GPU parity of the pseudofermion force hub_force and the autograd binding."""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import TINY, SMALL, DIFF_SUB, PREC, draw_inputs, draw_complex
from gpu_common import dev, to_dev, to_np, oracle_op, assert_close_elementwise

pytestmark = pytest.mark.gpu


def _hub(w, nrhs=1, path="auto"):
    from paper_2210_06874_amd import Hubbard
    return Hubbard(w.L, w.Nt, w.beta, w.kappa, nrhs_max=nrhs, path=path)


@pytest.mark.parametrize("path", ["fused", "split"])
@pytest.mark.parametrize("w", [TINY, DIFF_SUB, SMALL], ids=lambda w: w.name)
def test_force_kernel_matches_oracle_from_same_x(w, path):
    """hub_force(x) against the oracle's force from the same x (kernel alone)."""
    print(f"[case] force {w.name} {path}", flush=True)
    phi, x = draw_inputs(w, seed=21, nrhs=2)
    hub = _hub(w, nrhs=2, path=path)
    op = oracle_op(w)
    got = to_np(hub.force(to_dev(phi), to_dev(x)))
    assert_close_elementwise(got, O.force(op, phi, x), 1e-12, "force")


def test_force_precision_workload():
    w = PREC
    print(f"[case] force {w.name}", flush=True)
    phi, x = draw_inputs(w, seed=22)
    hub = _hub(w)
    op = oracle_op(w, mode="expm")
    got = to_np(hub.force(to_dev(phi), to_dev(x)))
    assert_close_elementwise(got, O.force(op, phi, x), 1e-12, "force")


def test_force_end_to_end_tiny_dense():
    """CG + force against the dense-oracle gradient; error bounded by cond * tol."""
    w = TINY
    phi, chi = draw_inputs(w)
    op = oracle_op(w)
    g_ref = O.force_dense(op, phi, O.dense_solve(op, phi, chi))
    hub = _hub(w)
    res = hub.cg_solve(to_dev(phi), to_dev(chi), tol=1e-13, max_iter=20000)
    g = to_np(hub.force(to_dev(phi), res.x))
    err = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    assert err < 1e-8, err


def test_autograd_backward_is_force():
    from paper_2210_06874_amd import PseudofermionAction
    w = TINY
    phi, chi = draw_inputs(w)
    hub = _hub(w)
    P = to_dev(phi).requires_grad_(True)
    S = PseudofermionAction.apply(P, to_dev(chi), hub, 1e-12)
    # what backward keeps: the field and the solution, nothing per slice
    saved = S.grad_fn.saved_tensors
    assert [tuple(t.shape) for t in saved] == [(w.Nt, w.V), (1, w.Nt, w.V)]
    S.backward()
    res = hub.cg_solve(to_dev(phi), to_dev(chi), tol=1e-12)
    g = hub.force(to_dev(phi), res.x)
    assert torch.equal(P.grad, g)
    op = oracle_op(w)
    x_ref = O.dense_solve(op, phi, chi)
    assert abs(S.item() - O.action(chi, x_ref)) <= 1e-9 * abs(S.item())
    # twice the same call: bitwise identical
    P2 = to_dev(phi).requires_grad_(True)
    S2 = PseudofermionAction.apply(P2, to_dev(chi), hub, 1e-12)
    S2.backward()
    assert S2.item() == S.item() and torch.equal(P2.grad, P.grad)


def test_autograd_gradient_in_chi():
    """d S / d chi: torch's gradient of a real function of complex chi is 2 dS/dchi^* = 2 x.
    Checked against the oracle's dense solve, and its convention against a central difference
    of the oracle's action along a random complex direction: dS = Re sum conj(grad) d."""
    from paper_2210_06874_amd import PseudofermionAction
    w = TINY
    print(f"[case] autograd chi {w.name}", flush=True)
    phi, chi = draw_inputs(w, nrhs=2)
    hub = _hub(w, nrhs=2)
    C = to_dev(chi).requires_grad_(True)
    P = to_dev(phi).requires_grad_(True)
    S = PseudofermionAction.apply(P, C, hub, 1e-12)
    S.backward()
    gc = to_np(C.grad)
    op = oracle_op(w)
    x_ref = O.dense_solve(op, phi, chi)
    cond = np.linalg.cond(op.dense_M(phi) @ op.dense_M(phi).conj().T)
    assert np.linalg.norm(gc - 2 * x_ref) <= 4 * cond * 1e-12 * np.linalg.norm(2 * x_ref)
    d = draw_complex(w, nrhs=2, seed=31)
    h = 1e-4
    Sp = O.action(chi + h * d, O.dense_solve(op, phi, chi + h * d))
    Sm = O.action(chi - h * d, O.dense_solve(op, phi, chi - h * d))
    fd = (Sp - Sm) / (2 * h)
    assert abs(fd - float(np.real(np.vdot(gc, d)))) <= 1e-6 * abs(fd)
    # phi's gradient is unchanged by also differentiating in chi
    assert torch.equal(P.grad, hub.force(to_dev(phi), hub.cg_solve(to_dev(phi), to_dev(chi), tol=1e-12).x))
    # a 2-D chi (one right-hand side) gets a 2-D gradient
    C1 = to_dev(chi[0]).requires_grad_(True)
    PseudofermionAction.apply(to_dev(phi), C1, _hub(w), 1e-12).backward()
    assert C1.grad.shape == C1.shape


def test_force_gauge_sum_rule_precision_workload():
    """sum_x g_{s-1,x} - sum_x g_{s,x} = -2 Im(chi_s^dag x_s) (P8) with x = hub's solution
    of a chi = M rho system on the weak-field L = 51 workload."""
    from workloads import draw_weak_field
    w = PREC
    phi, _ = draw_weak_field(w)
    rho = draw_complex(w, seed=3)
    hub = _hub(w)
    P = to_dev(phi)
    chi = hub.apply_M(P, to_dev(rho))
    res = hub.cg_solve(P, chi, tol=1e-12, max_iter=20000)
    assert res.converged
    g = to_np(hub.force(P, res.x))
    x = to_np(res.x)
    c = to_np(chi)
    lhs = np.roll(g.sum(axis=1), 1) - g.sum(axis=1)
    rhs = -2 * np.einsum("rtx,rtx->t", np.conj(c), x).imag
    scale = np.abs(g).sum(axis=1).max()
    np.testing.assert_allclose(lhs, rhs, atol=1e-9 * scale)


def test_cg_and_force_with_chemical_potential():
    """M[phi, mu] M[phi, mu]^dag stays Hermitian positive definite: CG and force at mu != 0
    against the oracle."""
    from paper_2210_06874_amd import Hubbard
    w = TINY
    mu = 0.4
    phi, chi = draw_inputs(w)
    op = O.HubbardOperator(w.L, w.Nt, w.beta, w.kappa, mu=mu)
    hub = Hubbard(w.L, w.Nt, w.beta, w.kappa, mu=mu)
    res = hub.cg_solve(to_dev(phi), to_dev(chi), tol=1e-12, max_iter=20000)
    x = to_np(res.x)
    assert np.linalg.norm(chi - op.apply_A(phi, x)) <= 2e-12 * np.linalg.norm(chi)
    g = to_np(hub.force(to_dev(phi), res.x))
    assert_close_elementwise(g, O.force(op, phi, x), 1e-12, "force")
    gd = O.force_dense(op, phi, O.dense_solve(op, phi, chi))
    assert np.linalg.norm(g - gd) <= 1e-7 * np.linalg.norm(gd)


def test_precision_workload_end_to_end():
    """L = 51, N_t = 128, weak field, heat-bath chi = M rho: the mixed-precision solve meets
    1e-10 on the residual the oracle recomputes, and its force is within 1e-8 of the
    oracle's force on an FP64 solution to 1e-12 (itself checked through M^dag x = rho)."""
    from workloads import draw_weak_field
    w = PREC
    print(f"[case] end to end {w.name}", flush=True)
    phi, _ = draw_weak_field(w)
    rho = draw_complex(w, seed=7)
    op = oracle_op(w, mode="expm")
    chi = op.apply_M(phi, rho)
    hub = _hub(w)
    P, C = to_dev(phi), to_dev(chi)
    mixed = hub.cg_solve(P, C, tol=1e-10, prec="mixed")
    tight = hub.cg_solve(P, C, tol=1e-12, prec="fp64", max_iter=40000)
    assert mixed.converged and tight.converged
    xm, xt = to_np(mixed.x), to_np(tight.x)
    rr = np.linalg.norm(chi - op.apply_A(phi, xm)) / np.linalg.norm(chi)
    assert rr <= 1.01e-10, rr
    hb = np.linalg.norm(op.apply_Mdag(phi, xt) - rho) / np.linalg.norm(rho)
    assert hb <= 1e-9, hb
    g_ref = O.force(op, phi, xt)
    g = to_np(hub.force(P, mixed.x))
    err = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"    residual {rr:.2e}, heat bath {hb:.2e}, force error {err:.2e}", flush=True)
    assert err <= 1e-8, err


def test_autograd_against_finite_differences_differentiation_workload():
    """L = 24, N_t = 64, beta = 8 (weak field: the prior draws do not converge at beta = 8):
    the autograd backward (the adjoint force kernel) against central finite differences at
    eps = 1e-6 on 64 random entries, each difference free of cancellation.  phi_{t,z} enters
    M only through column (t, z) of block (t+1, t): M = M' + e^{i phi} u e^T with
    u = -B_{t+1} E[:, z] on slice t+1.  Hence, with x+- = (M+- M+-^dag)^{-1} chi and
    Delta = e^{i phi-} - e^{i phi+},
        S+ - S- = x+^dag (A- - A+) x- = Delta conj(u^dag x+) x-_{t,z} + conj(Delta) conj(x+_{t,z}) u^dag x-,
    and u^dag x = -e^{i phi_{t,z}} (x - M^dag x)_{t,z} (from the (t, z) entry of M^dag x).
    Every term is O(|x|^2 eps): no large quantities are subtracted.  x+- are solved on the
    device to 1e-13 and M^dag x+- applied there.  Bar: 1e-8 on the norm over the 64 entries."""
    from paper_2210_06874_amd import PseudofermionAction
    from workloads import DIFF, draw_weak_field, pick_entries
    w = DIFF
    print(f"[case] finite differences {w.name}", flush=True)
    phi, chi = draw_weak_field(w)
    hub = _hub(w)
    P = to_dev(phi).requires_grad_(True)
    C = to_dev(chi)
    S = PseudofermionAction.apply(P, C, hub, 1e-13)
    S.backward()
    g = to_np(P.grad).ravel()
    eps = 1e-6
    idx = pick_entries(w, 64)
    fd = np.empty(len(idx))
    for n, j in enumerate(idx):
        t, z = divmod(int(j), w.V)
        sides = {}
        for sgn in (+1, -1):
            ph = phi.copy()
            ph[t, z] += sgn * eps
            Pd = to_dev(ph)
            x = hub.cg_solve(Pd, C, tol=1e-13, max_iter=40000).x
            y = hub.apply_Mdag(Pd, x)
            xe = complex(to_np(x[0, t, z]))
            d = xe - complex(to_np(y[0, t, z]))
            sides[sgn] = (ph[t, z], xe, -np.exp(1j * ph[t, z]) * d)       # (phi, x_{t,z}, u^dag x)
        (pp, xp, up), (pm, xm, um) = sides[+1], sides[-1]
        delta = np.exp(1j * pm) - np.exp(1j * pp)
        dS = delta * np.conj(up) * xm + np.conj(delta) * np.conj(xp) * um
        fd[n] = dS.real / (2 * eps)
    err = np.linalg.norm(fd - g[idx]) / np.linalg.norm(g[idx])
    print(f"    finite-difference error {err:.2e} over {len(idx)} entries", flush=True)
    assert err <= 1e-8, err


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_force_end_to_end_dense_sub_instance(prec):
    """The 18-site torus at the differentiation workload's N_t = 64, beta = 8, U = 3.8: device
    CG + force against the dense-oracle gradient (Sec. 2 eq. "ferm_op", eq. "hamiltonian").
    chi = M rho is the heat bath an HMC force sees; the literal iid chi has its FP64
    attainable-accuracy floor near 1e-6 here (||A|| ||x|| >> ||chi|| at cond(M M^dag) ~ 6e10),
    where no solver meets a 1e-11 tolerance.  The forward error of any x is bounded by
    cond(A) times its relative residual, which the oracle recomputes; both the solution's and
    the force's errors must stay within that bound (the force is bilinear in x: twice it).
    Measured: FP64 solves land about 1e-7 from the dense solution, mixed-precision ones (whose
    FP32 iterations leave more of the residual in the lowest modes) about 1e-5, both far
    inside the bound (about 0.6 at a 1e-11 residual)."""
    w = DIFF_SUB
    print(f"[case] end-to-end dense sub-instance {prec}", flush=True)
    phi, _ = draw_inputs(w)
    rho = draw_complex(w, seed=3)
    op = oracle_op(w)
    M = op.dense_M(phi)
    A = M @ M.conj().T
    cond = np.linalg.cond(A)
    chi = op.apply_M(phi, rho)
    x_ref = np.linalg.solve(M.conj().T, rho.ravel()).reshape(rho.shape)       # x = M^{-dag} rho
    g_ref = O.force_dense(op, phi, x_ref)
    hub = _hub(w)
    res = hub.cg_solve(to_dev(phi), to_dev(chi), tol=1e-11, max_iter=200000, prec=prec, stall_updates=5)
    x = to_np(res.x)
    rres = np.linalg.norm(chi.ravel() - A @ x.ravel()) / np.linalg.norm(chi)
    ex = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
    g = to_np(hub.force(to_dev(phi), res.x))
    eg = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"cond(A) {cond:.3e}  iters {res.iters[0]}  residual {rres:.2e}  x err {ex:.2e}  force err {eg:.2e}",
          flush=True)
    assert rres <= 2e-11
    assert ex <= cond * rres and eg <= 2 * cond * rres
    if prec == "fp64":
        assert eg <= 1e-6
