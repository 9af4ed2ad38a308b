"""Large-volume stress workload: L = 102 (20,808 sites, the paper's largest lattice),
Nt = 192, beta = 12, four right-hand sides solved together (the polynomial stencils in both
precisions; the context's transform layout, for the operators that use one, is the split path)."""
import numpy as np
import pytest
import torch

from workloads import STRESS, draw_weak_field, draw_complex
from gpu_common import dev, to_dev, to_np, oracle_op, assert_close_elementwise

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stress():
    from paper_2210_06874_amd import Hubbard
    w = STRESS
    hub = Hubbard(w.L, w.Nt, w.beta, w.kappa, nrhs_max=4)
    assert hub.path == "split"
    op = oracle_op(w, mode="expm")
    phi, _ = draw_weak_field(w)
    rho = draw_complex(w, nrhs=4, seed=9)
    P = to_dev(phi)
    chi = hub.apply_M(P, to_dev(rho))
    return w, hub, op, phi, rho, P, chi


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_stress_cg_heat_bath(stress, prec):
    """chi = M rho for 4 rhs at once: the oracle recomputes the true residual, and
    M^dag x = rho (Sec. 2 heat bath) for every right-hand side."""
    w, hub, op, phi, rho, P, chi = stress
    print(f"[case] stress cg {prec}", flush=True)
    res = hub.cg_solve(P, chi, tol=1e-10, prec=prec, max_iter=20000)
    assert res.converged, (res.true_rel_res, res.iters)
    x = to_np(res.x)
    c = to_np(chi)
    r = c - op.apply_A(phi, x)
    for k in range(4):
        rel = np.linalg.norm(r[k]) / np.linalg.norm(c[k])
        assert rel <= 2e-10, (k, rel)
        y = op.apply_Mdag(phi, x[k:k + 1])[0]
        assert np.linalg.norm(y - rho[k]) <= 1e-6 * np.linalg.norm(rho[k])


@pytest.mark.parametrize("persistent", [False, True])
def test_stress_batched_equals_single(stress, persistent):
    """The 4-rhs launch does per-rhs arithmetic identical to a 1-rhs solve, with two launches per
    iteration and with the persistent launch (every right-hand side's FP32 iterations in one
    cooperative launch per block of iterations)."""
    w, hub, op, phi, rho, P, chi = stress
    try:
        hub.set_cg_launch(persistent=persistent)
        res4 = hub.cg_solve(P, chi, tol=1e-10, prec="mixed", max_iter=20000)
        res1 = hub.cg_solve(P, chi[2:3].contiguous(), tol=1e-10, prec="mixed", max_iter=20000)
    finally:
        hub.set_cg_launch(persistent=False)
    assert (res4.persistent_launches > 0) == persistent and (res1.persistent_launches > 0) == persistent
    assert res4.iters[2] == res1.iters[0]
    assert torch.equal(res4.x[2], res1.x[0])


def test_stress_persistent_equals_two_kernel_iterations(stress):
    """The persistent launch (grid barriers between the M^dag and M phases) and two launches per
    iteration of the same sublattice kernel give the same solution bit for bit, with the same
    iteration counts."""
    w, hub, op, phi, rho, P, chi = stress
    print("[case] stress persistent vs two-kernel", flush=True)
    try:
        hub.set_cg_launch(sublattice=True)
        two = hub.cg_solve(P, chi, tol=1e-10, prec="mixed", max_iter=20000)
        hub.set_cg_launch(persistent=True)
        per = hub.cg_solve(P, chi, tol=1e-10, prec="mixed", max_iter=20000)
    finally:
        hub.set_cg_launch(persistent=False)
    assert two.persistent_launches == 0 and per.persistent_launches > 0
    assert two.iters == per.iters
    assert torch.equal(two.x, per.x)


def test_stress_persistent_barrier_wait_gives_up(stress):
    """A grid-barrier wait bounded to a single poll (forced from the host) runs out: every
    workgroup leaves the launch and the solve returns HUB_ERR_DEVICE; the next solve, with the
    default bound, is unaffected."""
    from paper_2210_06874_amd import HubError
    w, hub, op, phi, rho, P, chi = stress
    print("[case] stress persistent barrier give-up", flush=True)
    try:
        hub.set_cg_launch(persistent=True, barrier_spin_limit=1)
        with pytest.raises(HubError, match="HUB_ERR_DEVICE"):
            hub.cg_solve(P, chi, tol=1e-10, prec="mixed", max_iter=100)
        hub.set_cg_launch(persistent=True, barrier_spin_limit=0)
        res = hub.cg_solve(P, chi, tol=1e-10, prec="mixed", max_iter=20000)
    finally:
        hub.set_cg_launch(persistent=False)
    assert res.converged and res.persistent_launches > 0


def test_stress_force(stress):
    """hub_force summed over 4 rhs: against the oracle's force from the same x on sampled
    slices, and the gauge sum rule over every slice."""
    w, hub, op, phi, rho, P, chi = stress
    print("[case] stress force", flush=True)
    res = hub.cg_solve(P, chi, tol=1e-10, prec="mixed", max_iter=20000)
    g = to_np(hub.force(P, res.x))
    x = to_np(res.x)
    # sampled slices: g_t needs x_t and E x_{t+1}
    Bn = np.roll(op.B, -1)
    for t in (0, 95, w.Nt - 1):
        tn = (t + 1) % w.Nt
        wv = op.apply_E(x[:, tn])
        y = x[:, t] - Bn[t] * np.exp(-1j * phi[t])[None] * wv
        ref = (-2.0 * (-Bn[t] * 1j * np.exp(1j * phi[t])[None] * y * np.conj(wv)).real).sum(axis=0)
        assert_close_elementwise(g[t], ref, 1e-11, f"force slice {t}")
    c = to_np(chi)
    lhs = np.roll(g.sum(axis=1), 1) - g.sum(axis=1)
    rhs = -2 * np.einsum("rtx,rtx->t", np.conj(c), x).imag
    scale = np.abs(g).sum(axis=1).max()
    np.testing.assert_allclose(lhs, rhs, atol=1e-9 * scale)
