"""GPU parity of the time-slab entry points (hub_apply_M_slab, hub_apply_Mdag_slab, their FP32
variants and hub_force_slab): one shard of a time-sharded vector, nt consecutive slices with the
slice beyond each edge passed in as a halo, against the oracle's rows of the full operator."""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import PREC, STRESS, SMALL, Lattice, draw_inputs
from gpu_common import dev, to_dev, to_np, oracle_op, assert_close_elementwise

pytestmark = pytest.mark.gpu

RTOL64, RTOL32 = 1e-12, 2e-5


def _shard(a, t0, nt):
    """Slices t0 .. t0+nt-1 of [.., Nt, V] (a copy, as a shard would hold it)."""
    return np.ascontiguousarray(a[..., t0:t0 + nt, :])


def _slab_outputs(hub, phi, v, t0, nt, prec="fp64"):
    Nt = phi.shape[0]
    tp, tn = (t0 - 1) % Nt, (t0 + nt) % Nt
    rd, cd = (np.float64, np.complex128) if prec == "fp64" else (np.float32, np.complex64)
    P, Vs = to_dev(_shard(phi, t0, nt).astype(rd)), to_dev(_shard(v, t0, nt).astype(cd))
    ph_h = to_dev(np.ascontiguousarray(phi[tp]).astype(rd))
    vp = to_dev(np.ascontiguousarray(v[:, tp]).astype(cd))
    vn = to_dev(np.ascontiguousarray(v[:, tn]).astype(cd))
    if prec == "fp64":
        return (to_np(hub.apply_M_slab(t0, P, Vs, ph_h, vp)), to_np(hub.apply_Mdag_slab(t0, P, Vs, vn)),
                to_np(hub.force_slab(t0, P, Vs, vn)))
    return to_np(hub.apply_M_slab_c64(t0, P, Vs, ph_h, vp)), to_np(hub.apply_Mdag_slab_c64(t0, P, Vs, vn)), None


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_shards_of_the_precision_workload(prec):
    """L = 51, N_t = 128 cut into four shards of 32 slices (and one of a single slice at each
    wrap): every row of each shard's M, M^dag (and FP64 force) against the oracle's full rows."""
    from paper_2210_06874_amd import Hubbard
    w = PREC
    print(f"[case] slabs {w.name} {prec}", flush=True)
    phi, v = draw_inputs(w, seed=51)
    if prec == "fp32":
        phi = phi.astype(np.float32).astype(np.float64)
        v = v.astype(np.complex64).astype(np.complex128)
    op = oracle_op(w, mode="expm")
    M, D = op.apply_M(phi, v), op.apply_Mdag(phi, v)
    g = O.force(op, phi, v) if prec == "fp64" else None
    hub = Hubbard(w.L, w.Nt, w.beta, w.kappa)
    tol = RTOL64 if prec == "fp64" else RTOL32
    for t0, nt in [(0, 32), (32, 32), (64, 32), (96, 32), (0, 1), (w.Nt - 1, 1), (5, 70)]:
        gm, gd, gf = _slab_outputs(hub, phi, v, t0, nt, prec)
        assert_close_elementwise(gm, M[:, t0:t0 + nt], tol, f"M slab {t0}+{nt}")
        assert_close_elementwise(gd, D[:, t0:t0 + nt], tol, f"Mdag slab {t0}+{nt}")
        if gf is not None:
            assert_close_elementwise(gf, g[t0:t0 + nt], 1e-12, f"force slab {t0}+{nt}")


def test_whole_lattice_slab_reproduces_the_full_calls():
    """t0 = 0, nt = N_t, halos taken from the vector itself: the slab calls give hub_apply_M,
    hub_apply_Mdag and hub_force (2 right-hand sides)."""
    from paper_2210_06874_amd import Hubbard
    w = SMALL
    phi, v = draw_inputs(w, seed=52, nrhs=2)
    hub = Hubbard(w.L, w.Nt, w.beta, w.kappa, nrhs_max=2)
    gm, gd, gf = _slab_outputs(hub, phi, v, 0, w.Nt)
    P, V = to_dev(phi), to_dev(v)
    assert_close_elementwise(gm, to_np(hub.apply_M(P, V)), 1e-14, "M")
    assert_close_elementwise(gd, to_np(hub.apply_Mdag(P, V)), 1e-14, "Mdag")
    assert_close_elementwise(gf, to_np(hub.force(P, V)), 1e-14, "force")


def test_shards_of_the_stress_workload_sampled():
    """L = 102, N_t = 192, four right-hand sides: shards of 48 slices (the first, whose M halo
    wraps, and the last, whose M^dag and force halos wrap), FP64 and FP32 (the degree-9 and
    degree-5 polynomial stencils), on each shard's edge slices against the oracle."""
    from paper_2210_06874_amd import Hubbard
    w = STRESS
    print(f"[case] slabs {w.name}", flush=True)
    phi, v = draw_inputs(w, seed=53, nrhs=w.nrhs)
    op = oracle_op(w, mode="expm")
    hub = Hubbard(w.L, w.Nt, w.beta, w.kappa, nrhs_max=w.nrhs)
    for t0 in (0, 144):
        nt = 48
        for prec in ("fp64", "fp32"):
            ph = phi if prec == "fp64" else phi.astype(np.float32).astype(np.float64)
            vv = v if prec == "fp64" else v.astype(np.complex64).astype(np.complex128)
            gm, gd, gf = _slab_outputs(hub, ph, vv, t0, nt, prec)
            tol = RTOL64 if prec == "fp64" else RTOL32
            for tl in (0, nt - 1):
                t = t0 + tl
                tp, tn = (t - 1) % w.Nt, (t + 1) % w.Nt
                Bt, Btn = (-1.0 if t == 0 else 1.0), (-1.0 if tn == 0 else 1.0)
                wv = op.apply_E(vv[:, tn])
                assert_close_elementwise(gm[:, tl], vv[:, t] - Bt * op.apply_E(np.exp(1j * ph[tp])[None] * vv[:, tp]),
                                         tol, f"{prec} M row {t}")
                assert_close_elementwise(gd[:, tl], vv[:, t] - Btn * np.exp(-1j * ph[t])[None] * wv, tol,
                                         f"{prec} Mdag row {t}")
                if gf is not None:
                    gref = (-2.0 * Btn * (np.exp(1j * ph[t])[None] * vv[:, t] * np.conj(wv)).imag).sum(axis=0)
                    assert_close_elementwise(gf[tl], gref, 1e-11, f"force row {t}")


def test_slab_arguments_are_checked():
    from paper_2210_06874_amd import Hubbard, HubError
    w = Lattice("L3_Nt8", 3, 8, 2.0, 3.0)
    phi, v = draw_inputs(w)
    hub = Hubbard(w.L, w.Nt, w.beta, w.kappa)
    P, V = to_dev(phi), to_dev(v)
    h = to_dev(v[:, 0].copy())
    with pytest.raises(ValueError):
        hub.apply_M_slab(6, P[:4].contiguous(), V[:, :4].contiguous(), P[0].contiguous(), h)   # 6 + 4 > 8
    lib = hub.lib
    import ctypes
    p = ctypes.c_void_p
    # through the C ABI: slab past the end, empty slab, negative t0, NULL halo
    out = torch.empty_like(V)
    for t0, nt in ((6, 4), (0, 0), (-1, 2)):
        assert lib.hub_apply_Mdag_slab(hub._h, t0, nt, p(P.data_ptr()), p(V.data_ptr()), p(h.data_ptr()),
                                       p(out.data_ptr()), 1, None) == 1
    assert lib.hub_apply_Mdag_slab(hub._h, 0, 8, p(P.data_ptr()), p(V.data_ptr()), None,
                                   p(out.data_ptr()), 1, None) == 1
    lin = Hubbard(w.L, w.Nt, w.beta, w.kappa, form="linear")
    with pytest.raises(HubError):
        lin.apply_Mdag_slab(0, P, V, h)
