"""A seeded sweep over random small problems: both forms, the fused and split paths, mu != 0,
one to four right-hand sides, delta*kappa between -1 and 1.  Every case checks M and M^dag in FP64,
M in FP32, the force on random vectors and, for the smaller ones, a mixed-precision solve, all
against the oracle."""
import numpy as np
import pytest

import oracle as O
from workloads import Lattice, draw_phi, draw_complex
from gpu_common import dev, to_dev, to_np, assert_close_elementwise

pytestmark = pytest.mark.gpu

# lengths whose prime factors the transforms support (<= 17), and any length for the stencil
_FFT_L = [L for L in range(1, 61) if all(p <= 17 for p in range(2, L + 1)
                                         if L % p == 0 and all(p % q for q in range(2, p)))]


def _cases(n=60, seed=2718):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        form = "linear" if rng.random() < 0.3 else "exp"
        L = int(rng.choice(_FFT_L)) if form == "exp" else int(rng.integers(1, 48))
        Nt = int(rng.integers(1, 40))
        beta = float(rng.uniform(0.2, 8.0))
        kmax = min(2.5, Nt / beta)                                 # |delta * kappa| <= 1
        kappa = float(rng.uniform(-kmax, kmax))
        mu = float(rng.uniform(-0.8, 0.8)) if form == "exp" and rng.random() < 0.3 else 0.0
        path = "split" if form == "exp" and rng.random() < 0.3 else "auto"
        out.append((form, L, Nt, int(rng.integers(1, 5)), beta, kappa, mu, path))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: "{}-L{}-Nt{}-r{}-{}".format(c[0], c[1], c[2], c[3], c[7]))
def test_random_shape_against_oracle(case):
    from paper_2210_06874_amd import Hubbard
    form, L, Nt, nrhs, beta, kappa, mu, path = case
    print(f"[case] {case}", flush=True)
    w = Lattice(f"L{L}_Nt{Nt}", L, Nt, beta, 3.0, kappa=kappa, nrhs=nrhs)
    rng = np.random.default_rng(L * 1000 + Nt)
    phi = draw_phi(w, rng=rng)
    v = draw_complex(w, nrhs=nrhs, rng=rng)
    op = O.LinearHubbardOperator(L, Nt, beta, kappa) if form == "linear" else O.HubbardOperator(L, Nt, beta, kappa, mu=mu)
    hub = Hubbard(L, Nt, beta, kappa, nrhs_max=nrhs, path=path, form=form, mu=mu)
    P, Vd = to_dev(phi), to_dev(v)
    assert_close_elementwise(to_np(hub.apply_M(P, Vd)), op.apply_M(phi, v), 1e-12, "M")
    assert_close_elementwise(to_np(hub.apply_Mdag(P, Vd)), op.apply_Mdag(phi, v), 1e-12, "Mdag")
    p32, v32 = phi.astype(np.float32), v.astype(np.complex64)
    assert_close_elementwise(to_np(hub.apply_M_c64(to_dev(p32), to_dev(v32))),
                             op.apply_M(p32.astype(np.float64), v32.astype(np.complex128)), 2e-5, "M32")
    g_ref = O.force_linear(op, phi, v) if form == "linear" else O.force(op, phi, v)
    assert_close_elementwise(to_np(hub.force(P, Vd)), g_ref, 1e-11, "force")
    if w.N <= 4000:
        chi = op.apply_M(phi, v)
        res = hub.cg_solve(P, to_dev(chi), tol=1e-10, prec="mixed", max_iter=50000)
        r = chi - op.apply_A(phi, to_np(res.x))
        for k in range(nrhs):
            assert np.linalg.norm(r[k]) <= 2e-10 * np.linalg.norm(chi[k])
    hub.close()
