"""GPU parity on the HMC-generated L = 51, Nt = 128 field (Sec. 2: the fields an HMC force
sees carry the weight det(M M^dag), unlike the Gaussian prior draws, on which M M^dag is too
ill-conditioned for CG).  The field is an input like any other: every expected value below
comes from the oracle applied to it."""
import numpy as np
import pytest

import oracle as O
from workloads import PREC, draw_complex, load_hmc_field
from gpu_common import to_dev, to_np, oracle_op

pytestmark = pytest.mark.gpu


def test_hmc_field_solve_and_force_against_oracle():
    """Heat-bath chi = M rho on the stored HMC field: the mixed-precision solve to 1e-10 meets
    1e-10 on the residual the oracle recomputes; an FP64 solve to 1e-12 satisfies M^dag x = rho
    (the heat-bath identity, checked by the oracle) and its force is within 1e-12 of the
    oracle's force on that x (the kernel).  On this field a 1e-10 residual bounds x only to
    cond(M M^dag) * 1e-10, and the mixed force after the 1e-10 solve is ~2e-7 from the oracle's;
    the force of a mixed solve to 1e-12 meets the 1e-8 bar."""
    from paper_2210_06874_amd import Hubbard
    w = PREC
    print(f"[case] HMC field {w.name}", flush=True)
    phi, meta = load_hmc_field()
    assert phi.shape == (w.Nt, w.V) and meta["U"] == w.U and meta["beta"] == w.beta
    rho = draw_complex(w, seed=11)
    op = oracle_op(w, mode="expm")
    chi = op.apply_M(phi, rho)
    hub = Hubbard(w.L, w.Nt, w.beta, w.kappa)
    P, C = to_dev(phi), to_dev(chi)
    mixed = hub.cg_solve(P, C, tol=1e-10, prec="mixed", max_iter=100000)
    tight = hub.cg_solve(P, C, tol=1e-12, prec="fp64", max_iter=100000)
    assert mixed.converged and tight.converged, (mixed.true_rel_res, tight.true_rel_res)
    xm, xt = to_np(mixed.x), to_np(tight.x)
    rr = np.linalg.norm(chi - op.apply_A(phi, xm)) / np.linalg.norm(chi)
    assert rr <= 1.01e-10, rr
    hb = np.linalg.norm(op.apply_Mdag(phi, xt) - rho) / np.linalg.norm(rho)
    assert hb <= 1e-8, hb
    g_ref = O.force(op, phi, xt)
    g_t = to_np(hub.force(P, tight.x))
    kern = np.linalg.norm(g_t - g_ref) / np.linalg.norm(g_ref)
    assert kern <= 1e-12, kern
    g = to_np(hub.force(P, mixed.x))
    err10 = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    assert err10 <= 1e-6, err10
    mixed12 = hub.cg_solve(P, C, tol=1e-12, prec="mixed", max_iter=100000)
    assert mixed12.converged, mixed12.true_rel_res
    g12 = to_np(hub.force(P, mixed12.x))
    err = np.linalg.norm(g12 - g_ref) / np.linalg.norm(g_ref)
    print(f"    iterations mixed {mixed.iters[0]} (1e-12: {mixed12.iters[0]}) / fp64 {tight.iters[0]}, "
          f"residual {rr:.2e}, heat bath {hb:.2e}, force kernel {kern:.2e}, force error after the "
          f"1e-10 solve {err10:.2e}, after the 1e-12 solve {err:.2e}", flush=True)
    assert err <= 1e-8, err
