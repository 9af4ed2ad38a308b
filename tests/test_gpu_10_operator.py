"""GPU parity of the fermion operator kernels (hub_apply_M / hub_apply_Mdag and their
FP32 variants) against the FP64 CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import TINY, SMALL, DIFF, PREC, STRESS, Lattice, draw_inputs, draw_complex
from gpu_common import dev, to_dev, to_np, oracle_op, assert_close_elementwise
import closed_forms as CF

pytestmark = pytest.mark.gpu

RTOL64 = 1e-12     # FP64: transform roundoff ~ (stages) * 2^-53 relative to the largest entry
RTOL32 = 2e-5      # FP32: the same arithmetic at 2^-24


def _hub(w, path="auto", nrhs=1):
    from paper_2210_06874_amd import Hubbard
    return Hubbard(w.L, w.Nt, w.beta, w.kappa, nrhs_max=nrhs, path=path)


EDGE = [
    Lattice("L1_Nt1", 1, 1, 0.5, 3.0), Lattice("L1_Nt2", 1, 2, 1.0, 3.0),
    Lattice("L2_Nt2", 2, 2, 0.7, 3.0), Lattice("L5_Nt3", 5, 3, 1.5, 3.0),
    Lattice("L7_Nt4", 7, 4, 2.0, 3.0), Lattice("L10_Nt5", 10, 5, 2.0, 3.0),
    Lattice("L17_Nt3", 17, 3, 1.0, 3.0), Lattice("L6_Nt9", 6, 9, 3.0, 3.0),
]


@pytest.mark.parametrize("path", ["fused", "split"])
@pytest.mark.parametrize("w", [TINY, SMALL] + EDGE, ids=lambda w: w.name)
def test_apply_fp64_matches_oracle(w, path):
    print(f"[case] apply fp64 {w.name} path={path}", flush=True)
    phi, v = draw_inputs(w, seed=11, nrhs=2)
    hub = _hub(w, path, nrhs=2)
    assert hub.path == path
    op = oracle_op(w)
    got_M = to_np(hub.apply_M(to_dev(phi), to_dev(v)))
    got_D = to_np(hub.apply_Mdag(to_dev(phi), to_dev(v)))
    assert_close_elementwise(got_M, op.apply_M(phi, v), RTOL64, "M")
    assert_close_elementwise(got_D, op.apply_Mdag(phi, v), RTOL64, "Mdag")


@pytest.mark.parametrize("path", ["fused", "split"])
@pytest.mark.parametrize("w", [TINY, SMALL, EDGE[3], EDGE[6]], ids=lambda w: w.name)
def test_apply_fp32_matches_oracle(w, path):
    print(f"[case] apply fp32 {w.name} path={path}", flush=True)
    phi, v = draw_inputs(w, seed=12)
    phi32 = phi.astype(np.float32)
    v64 = v.astype(np.complex64)
    hub = _hub(w, path)
    op = oracle_op(w)
    ref_M = op.apply_M(phi32.astype(np.float64), v64.astype(np.complex128))
    ref_D = op.apply_Mdag(phi32.astype(np.float64), v64.astype(np.complex128))
    got_M = to_np(hub.apply_M_c64(to_dev(phi32), to_dev(v64)))
    got_D = to_np(hub.apply_Mdag_c64(to_dev(phi32), to_dev(v64)))
    assert_close_elementwise(got_M, ref_M, RTOL32, "M32")
    assert_close_elementwise(got_D, ref_D, RTOL32, "Mdag32")


def test_apply_diff_workload_fp64():
    w = DIFF
    print(f"[case] apply fp64 {w.name}", flush=True)
    phi, v = draw_inputs(w, seed=13)
    hub = _hub(w)
    op = oracle_op(w, mode="expm")
    assert_close_elementwise(to_np(hub.apply_M(to_dev(phi), to_dev(v))), op.apply_M(phi, v), RTOL64, "M")
    assert_close_elementwise(to_np(hub.apply_Mdag(to_dev(phi), to_dev(v))), op.apply_Mdag(phi, v), RTOL64, "Mdag")


@pytest.mark.parametrize("prec,path", [("fp64", "auto"), ("fp32", "auto"), ("fp32", "fused")])
def test_apply_precision_workload(prec, path):
    """L = 51, Nt = 128: the full operator against the oracle's Krylov-exp route (FP32: the
    default polynomial-stencil kernel and the transform kernels of the forced fused path)."""
    w = PREC
    print(f"[case] apply {prec} {w.name} path={path}", flush=True)
    phi, v = draw_inputs(w, seed=14)
    hub = _hub(w, path=path)
    op = oracle_op(w, mode="expm")
    if prec == "fp64":
        got = to_np(hub.apply_M(to_dev(phi), to_dev(v)))
        assert_close_elementwise(got, op.apply_M(phi, v), RTOL64, "M")
        got = to_np(hub.apply_Mdag(to_dev(phi), to_dev(v)))
        assert_close_elementwise(got, op.apply_Mdag(phi, v), RTOL64, "Mdag")
    else:
        p32, v32 = phi.astype(np.float32), v.astype(np.complex64)
        got = to_np(hub.apply_M_c64(to_dev(p32), to_dev(v32)))
        ref = op.apply_M(p32.astype(np.float64), v32.astype(np.complex128))
        assert_close_elementwise(got, ref, RTOL32, "M32")
        got = to_np(hub.apply_Mdag_c64(to_dev(p32), to_dev(v32)))
        ref = op.apply_Mdag(p32.astype(np.float64), v32.astype(np.complex128))
        assert_close_elementwise(got, ref, RTOL32, "Mdag32")


@pytest.mark.parametrize("path", ["auto", "fused"])
@pytest.mark.parametrize("nrhs", [1, 2])
def test_apply_fp32_both_operators_precision_workload(nrhs, path):
    """L = 51, N_t = 128 in FP32: M and M^dag, every entry, with one and two right-hand sides,
    against the oracle applied to the same FP32-rounded inputs.  path auto: the polynomial-stencil
    kernel (two workgroups per slice, each writing half the columns); fused: the transform
    kernels (one right-hand side, 128 slices: two workgroups per slice, each writing one
    sublattice; two, 256 slices: one workgroup per slice)."""
    w = PREC
    print(f"[case] apply fp32 M and Mdag {w.name} nrhs={nrhs} path={path}", flush=True)
    phi, v = draw_inputs(w, seed=24, nrhs=nrhs)
    hub = _hub(w, nrhs=nrhs, path=path)
    op = oracle_op(w, mode="expm")
    p32, v32 = phi.astype(np.float32), v.astype(np.complex64)
    p64, v64 = p32.astype(np.float64), v32.astype(np.complex128)
    P, V = to_dev(p32), to_dev(v32)
    assert_close_elementwise(to_np(hub.apply_M_c64(P, V)), op.apply_M(p64, v64), RTOL32, "M32")
    assert_close_elementwise(to_np(hub.apply_Mdag_c64(P, V)), op.apply_Mdag(p64, v64), RTOL32, "Mdag32")


@pytest.mark.parametrize("w", [TINY, SMALL, PREC], ids=lambda w: w.name)
def test_negative_kappa_and_the_hole_operator(w):
    """kappa = -1: M, M^dag (FP64 and FP32) and the force against the oracle, and the hole
    operator M[-phi, -kappa] of the weight det(M M^dag) (Sec. 2).  A negative delta*kappa
    exercises every branch of the E(k) table."""
    from paper_2210_06874_amd import Hubbard
    print(f"[case] negative kappa {w.name}", flush=True)
    phi, v = draw_inputs(w, seed=25)
    mode = "expm" if w.L > 20 else None
    for sgn in (1.0, -1.0):                        # M[phi, -1] and the hole operator M[-phi, -1]
        ph = sgn * phi
        op = O.HubbardOperator(w.L, w.Nt, w.beta, -1.0, mode=mode)
        hub = Hubbard(w.L, w.Nt, w.beta, -1.0)
        P, V = to_dev(ph), to_dev(v)
        assert_close_elementwise(to_np(hub.apply_M(P, V)), op.apply_M(ph, v), RTOL64, f"M sgn={sgn}")
        assert_close_elementwise(to_np(hub.apply_Mdag(P, V)), op.apply_Mdag(ph, v), RTOL64, f"Mdag sgn={sgn}")
        p32, v32 = ph.astype(np.float32), v.astype(np.complex64)
        p64, v64 = p32.astype(np.float64), v32.astype(np.complex128)
        assert_close_elementwise(to_np(hub.apply_M_c64(to_dev(p32), to_dev(v32))), op.apply_M(p64, v64), RTOL32,
                                 f"M32 sgn={sgn}")
        assert_close_elementwise(to_np(hub.apply_Mdag_c64(to_dev(p32), to_dev(v32))), op.apply_Mdag(p64, v64),
                                 RTOL32, f"Mdag32 sgn={sgn}")
        assert_close_elementwise(to_np(hub.force(P, V)), O.force(op, ph, v), 1e-12, f"force sgn={sgn}")
        hub.close()


def _stress_slices(op, phi, v, slices, dagger):
    """Oracle rows of M v (or M^dag v) for a few destination slices only."""
    out = {}
    for t in slices:
        if not dagger:
            ts = (t - 1) % op.Nt
            src = np.exp(1j * phi[ts])[None] * v[:, ts]
            hop = op.apply_E(src)
            out[t] = v[:, t] - op.B[t] * hop
        else:
            ts = (t + 1) % op.Nt
            hop = op.apply_E(v[:, ts])
            out[t] = v[:, t] - op.B[ts] * np.exp(-1j * phi[t])[None] * hop
    return out


# the sublattice kernel is FP32 only
@pytest.mark.parametrize("prec,kernel", [("fp64", "default"), ("fp64", "split"), ("fp32", "default"),
                                         ("fp32", "sublattice"), ("fp32", "split")])
def test_apply_stress_workload_sampled(prec, kernel):
    """L = 102, Nt = 192, 4 right-hand sides in one call: sampled slices, including both wrap
    slices, against the oracle (the default polynomial stencil, degree 9 in FP64 and 5 in FP32;
    the forced split path; the FP32 sublattice kernel)."""
    w = STRESS
    print(f"[case] apply {prec} {w.name} {kernel}", flush=True)
    phi, v = draw_inputs(w, seed=15)
    hub = _hub(w, nrhs=4, path="split" if kernel == "split" else "auto")
    if kernel == "sublattice":
        hub.set_cg_launch(sublattice=True)
    op = oracle_op(w, mode="expm")
    slices = [0, 1, 77, w.Nt - 1]
    if prec == "fp32":
        phi = phi.astype(np.float32).astype(np.float64)
        v = v.astype(np.complex64).astype(np.complex128)
        gM = to_np(hub.apply_M_c64(to_dev(phi.astype(np.float32)), to_dev(v.astype(np.complex64))))
        gD = to_np(hub.apply_Mdag_c64(to_dev(phi.astype(np.float32)), to_dev(v.astype(np.complex64))))
        tol = RTOL32
    else:
        gM = to_np(hub.apply_M(to_dev(phi), to_dev(v)))
        gD = to_np(hub.apply_Mdag(to_dev(phi), to_dev(v)))
        tol = RTOL64
    for dag, got in ((False, gM), (True, gD)):
        ref = _stress_slices(op, phi, v, slices, dag)
        for t in slices:
            assert_close_elementwise(got[:, t], ref[t], tol, f"slice {t} dag={dag}")


@pytest.mark.parametrize("mu,kappa", [(0.0, 1.0), (0.3, 1.0), (0.0, -1.0)])
def test_fp64_stencil_and_split_path_agree_at_L102(mu, kappa):
    """The FP64 operators and the force at L = 102 by the degree-9 polynomial stencil (default)
    and by the split-path transforms, on every entry of 4 right-hand sides: both are
    E = e^{delta mu} exp(delta kappa K) to FP64 accuracy (the series' bound is 2.9e-17 at this
    step, Sec. 2 eq. "ferm_op"; mu enters as the scale, a negative kappa through the sweeps'
    coefficients), so they agree to the transforms' rounding.  The oracle checks both on sampled
    slices at mu = 0, kappa = 1."""
    from paper_2210_06874_amd import Hubbard
    w = STRESS
    print(f"[case] fp64 stencil vs split {w.name} mu={mu} kappa={kappa}", flush=True)
    phi, v = draw_inputs(w, seed=18)
    P, V = to_dev(phi), to_dev(v)
    poly = Hubbard(w.L, w.Nt, w.beta, kappa, nrhs_max=4, mu=mu)
    split = Hubbard(w.L, w.Nt, w.beta, kappa, nrhs_max=4, mu=mu, path="split")
    for f in ("apply_M", "apply_Mdag", "force"):
        a = to_np(getattr(poly, f)(P, V))
        b = to_np(getattr(split, f)(P, V))
        err = np.abs(a - b).max() / np.abs(b).max()
        assert err <= 1e-14, (f, err)
    poly.close()
    split.close()


@pytest.mark.parametrize("w", [PREC, STRESS], ids=lambda w: w.name)
def test_adjointness_at_scale(w):
    """<u, M v> = <M^dag u, v> on the GPU at full size (P6)."""
    print(f"[case] adjointness {w.name}", flush=True)
    phi, u = draw_inputs(w, seed=16)
    vv = draw_complex(w, seed=17)
    hub = _hub(w, nrhs=w.nrhs)
    P, U, Vv = to_dev(phi), to_dev(u), to_dev(vv)
    a = torch.vdot(U.flatten(), hub.apply_M(P, Vv).flatten()).item()
    b = torch.vdot(hub.apply_Mdag(P, U).flatten(), Vv.flatten()).item()
    assert abs(a - b) <= 1e-11 * abs(a)


@pytest.mark.parametrize("w", [PREC, STRESS], ids=lambda w: w.name)
def test_free_plane_waves_at_scale(w):
    """phi = 0: plane waves are eigenvectors with eigenvalue 1 - e^{-i omega} e^{delta eps} (P2)."""
    print(f"[case] plane waves {w.name}", flush=True)
    hub = _hub(w)
    phi = torch.zeros((w.Nt, w.V), dtype=torch.float64, device=dev())
    for (n, m1, m2, band) in [(0, 0, 0, 1), (w.Nt - 1, w.L // 3, 2 * w.L // 3, -1), (5, 7, 11, 1)]:
        v, eps, om = CF.plane_wave(w.L, w.Nt, n, m1, m2, band)
        lam = CF.free_M_eigenvalue(eps, om, w.delta)
        got = to_np(hub.apply_M(phi, to_dev(v)))
        # relative to the input's scale: near omega ~ 2 pi the eigenvalue is small and
        # M v is a difference of two terms of size |v|
        err = np.abs(got - lam * v).max() / np.abs(v).max()
        assert err <= RTOL64, f"plane wave {n},{m1},{m2}: {err:.3e}"


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_half_and_whole_slice_kernels_agree(prec):
    """L = 51: one right-hand side runs two workgroups per slice (each writes one
    sublattice), two right-hand sides run one workgroup per slice; both match the oracle."""
    w = PREC
    print(f"[case] paired vs single {prec} {w.name}", flush=True)
    phi, v = draw_inputs(w, seed=18, nrhs=2)
    hub = _hub(w, nrhs=2, path="fused")
    op = oracle_op(w, mode="expm")
    if prec == "fp64":
        P, V = to_dev(phi), to_dev(v)
        one = [to_np(hub.apply_M(P, V[r:r + 1].contiguous())) for r in range(2)]
        two = to_np(hub.apply_M(P, V))
        ref = op.apply_M(phi, v)
        tol = RTOL64
    else:
        p32, v32 = phi.astype(np.float32), v.astype(np.complex64)
        P, V = to_dev(p32), to_dev(v32)
        one = [to_np(hub.apply_M_c64(P, V[r:r + 1].contiguous())) for r in range(2)]
        two = to_np(hub.apply_M_c64(P, V))
        ref = op.apply_M(p32.astype(np.float64), v32.astype(np.complex128))
        tol = RTOL32
    for r in range(2):
        assert_close_elementwise(one[r][0], ref[r], tol, f"half-slice kernel rhs {r}")
        assert_close_elementwise(two[r], ref[r], tol, f"whole-slice kernel rhs {r}")


@pytest.mark.parametrize("mu", [0.35, -0.6])
def test_apply_with_chemical_potential(mu):
    """mu != 0 (Sec. 3): every time hop carries e^{delta mu}; fused and L = 51 kernels."""
    from paper_2210_06874_amd import Hubbard
    for w in (SMALL, PREC):
        print(f"[case] apply mu={mu} {w.name}", flush=True)
        phi, v = draw_inputs(w, seed=19)
        hub = Hubbard(w.L, w.Nt, w.beta, w.kappa, mu=mu)
        op = O.HubbardOperator(w.L, w.Nt, w.beta, w.kappa, mode="expm", mu=mu)
        assert_close_elementwise(to_np(hub.apply_M(to_dev(phi), to_dev(v))), op.apply_M(phi, v), RTOL64, "M")
        assert_close_elementwise(to_np(hub.apply_Mdag(to_dev(phi), to_dev(v))), op.apply_Mdag(phi, v), RTOL64,
                                 "Mdag")


@pytest.mark.parametrize("dag", [False, True])
def test_sublattice_and_split_kernels_agree(dag):
    """L = 102 in FP32: the default polynomial-stencil kernel, the one-workgroup-per-slice kernel that
    keeps one sublattice's spectrum in registers (selected by the sublattice launch mode) and the
    three-kernel split path agree (all against the oracle on sampled slices in
    test_apply_stress_workload_sampled)."""
    w = STRESS
    print(f"[case] polynomial vs sublattice vs split dag={dag}", flush=True)
    phi, v = draw_inputs(w, seed=18, nrhs=2)
    P32, V32 = to_dev(phi.astype(np.float32)), to_dev(v.astype(np.complex64))
    a = _hub(w, "auto", nrhs=2)
    b = _hub(w, "split", nrhs=2)
    fa = a.apply_Mdag_c64 if dag else a.apply_M_c64
    fb = b.apply_Mdag_c64 if dag else b.apply_M_c64
    poly = to_np(fa(P32, V32))
    a.set_cg_launch(sublattice=True)
    sub = to_np(fa(P32, V32))
    a.set_cg_launch()
    split = to_np(fb(P32, V32))
    assert_close_elementwise(poly, split, 4e-6, "polynomial vs split")
    assert_close_elementwise(sub, split, 4e-6, "sub vs split")


@pytest.mark.parametrize("form", ["exp", "linear"])
def test_graph_replays_match_eager(form):
    """The operators captured in a HIP graph (the way the benchmark times them): every
    replay, with eager work and synchronisations between replays, equals the eager result
    bit for bit."""
    from paper_2210_06874_amd import Hubbard
    w = PREC
    print(f"[case] graph replays {form}", flush=True)
    phi, v = draw_inputs(w, seed=19)
    hub = Hubbard(w.L, w.Nt, w.beta, w.kappa, form=form)
    P32, V32 = to_dev(phi.astype(np.float32)), to_dev(v.astype(np.complex64))
    P, V = to_dev(phi), to_dev(v)
    eager32 = hub.apply_M_c64(P32, V32).clone()
    eager64 = hub.apply_Mdag(P, V).clone()
    out32, out64 = torch.empty_like(V32), torch.empty_like(V)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for _ in range(3):
                hub.apply_M_c64(P32, V32, out=out32)
                hub.apply_Mdag(P, V, out=out64)
    for rep in range(4):
        out32.zero_()
        out64.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out32, eager32), rep
        assert torch.equal(out64, eager64), rep
        hub.apply_M(P, V)                     # eager work between replays
        torch.cuda.synchronize()


def test_operators_on_a_side_stream():
    """Calls enqueue on the caller's current stream (here a side stream, default priority)."""
    w = SMALL
    phi, v = draw_inputs(w, seed=20)
    hub = _hub(w)
    P, V = to_dev(phi), to_dev(v)
    ref = hub.apply_M(P, V).clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        got = hub.apply_M(P, V)
        res = hub.cg_solve(P, V, tol=1e-8, prec="mixed")
    s.synchronize()
    assert torch.equal(got, ref)
    assert res.converged


MAXL = Lattice("L1024_Nt2", 1024, 2, 0.5, 3.0)      # the largest torus the ABI accepts


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_maximum_lattice(prec):
    """L = 1024 (2 M sites per slice, the split path with runtime radix-4 plans), every
    entry against the oracle's Krylov-exp route."""
    w = MAXL
    print(f"[case] apply {prec} {w.name}", flush=True)
    phi, v = draw_inputs(w, seed=21)
    hub = _hub(w)
    assert hub.path == "split"
    op = oracle_op(w, mode="expm")
    if prec == "fp64":
        got = to_np(hub.apply_M(to_dev(phi), to_dev(v)))
        ref = op.apply_M(phi, v)
        tol = RTOL64
    else:
        p32, v32 = phi.astype(np.float32), v.astype(np.complex64)
        got = to_np(hub.apply_M_c64(to_dev(p32), to_dev(v32)))
        ref = op.apply_M(p32.astype(np.float64), v32.astype(np.complex128))
        tol = RTOL32
    assert_close_elementwise(got, ref, tol, "M")


@pytest.mark.parametrize("form", ["exp", "linear"])
def test_kappa_zero_is_a_pure_time_hop(form):
    """kappa = 0 (degenerate: no spatial hopping, E = 1): every site is an independent
    antiperiodic time chain, written out here directly from the operator's definition."""
    from paper_2210_06874_amd import Hubbard
    w = SMALL
    phi, v = draw_inputs(w, seed=22)
    hub = Hubbard(w.L, w.Nt, w.beta, 0.0, form=form)
    got = to_np(hub.apply_M(to_dev(phi), to_dev(v)))[0]
    v0 = v[0]
    B = np.ones(w.Nt)
    B[0] = -1.0
    e = np.exp(1j * phi)
    prev = B[:, None] * np.roll(v0, 1, axis=0)              # B_t v_{t-1}
    if form == "exp":
        ref = v0 - B[:, None] * np.roll(e * v0, 1, axis=0)  # v_t - B_t e^{i phi_{t-1}} v_{t-1}
    else:
        nxt = np.roll(B, -1)[:, None] * np.roll(v0, -1, axis=0)   # B_{t+1} v_{t+1}
        LL = w.L * w.L
        ref = np.empty_like(v0)
        ref[:, :LL] = nxt[:, :LL] - e[:, :LL] * v0[:, :LL]
        ref[:, LL:] = v0[:, LL:] - np.conj(e[:, LL:]) * prev[:, LL:]
    assert_close_elementwise(got, ref, RTOL64, "kappa=0")


def test_output_buffers_are_checked():
    """The binding refuses an out tensor the kernels would overrun or misread (short, strided,
    wrong dtype or device) and writes a correct one in place, 2-D or 3-D."""
    from paper_2210_06874_amd import Hubbard
    w = TINY
    phi, v = draw_inputs(w)
    hub = Hubbard(w.L, w.Nt, w.beta, w.kappa)
    P, V = to_dev(phi), to_dev(v[0])
    ref = hub.apply_M(P, V)
    bad = [torch.empty((w.Nt, w.V - 1), dtype=torch.complex128, device=dev()),
           torch.empty((w.Nt, w.V), dtype=torch.complex64, device=dev()),
           torch.empty((w.V, w.Nt), dtype=torch.complex128, device=dev()).t(),
           torch.empty((w.Nt, w.V), dtype=torch.complex128)]
    for o in bad:
        with pytest.raises(ValueError):
            hub.apply_M(P, V, out=o)
    with pytest.raises(ValueError):
        hub.force(P, V, out=torch.empty((w.Nt, w.V), dtype=torch.float32, device=dev()))
    o2 = torch.empty_like(V)
    r2 = hub.apply_M(P, V, out=o2)
    assert r2.data_ptr() == o2.data_ptr() and torch.equal(o2, ref)
    o3 = torch.empty((1, w.Nt, w.V), dtype=torch.complex128, device=dev())
    with pytest.raises(ValueError):
        hub.apply_M(P, V, out=o3)            # out must have the input's own shape
    r3 = hub.apply_M(P, V[None], out=o3)
    assert r3.data_ptr() == o3.data_ptr() and torch.equal(o3[0], ref)
    g = torch.empty_like(P)
    assert hub.force(P, V, out=g).data_ptr() == g.data_ptr()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_phase_accuracy_over_the_angle_range(prec):
    """At kappa = 0 and v = 1, (M v)_t = 1 - B_t e^{i phi_{t-1}}, so the operator exposes every
    phase it evaluates.  Angles from 1e-3 to 2e7, multiples of pi/2 and values on both sides
    of the fast paths' limits (6,000 in FP32, 1e5 in FP64) must match e^{i phi} of the input
    as given: FP64 to a few ulp, FP32 to the rounding of its argument reduction
    (|phi| 2^-24 when |phi| < 6,000) plus the hardware sin/cos error."""
    from paper_2210_06874_amd import Hubbard
    w = Lattice("L3_Nt4", 3, 4, 1.0, 3.0, kappa=0.0)
    rng = np.random.default_rng(41)
    special = [0.0, np.pi / 2, -np.pi, 3 * np.pi / 2, 1e3 * np.pi, 5999.9, -6000.1, 6000.0,
               99999.9, -100000.1, 1e5, 2e7, -2e7, 1234567.89]
    mags = 10.0 ** rng.uniform(-3, 7.3, size=w.N - len(special))
    phi = np.concatenate([special, mags * rng.choice([-1.0, 1.0], size=mags.size)]).reshape(w.Nt, w.V)
    hub = Hubbard(w.L, w.Nt, w.beta, w.kappa)
    B = np.ones(w.Nt)
    B[0] = -1.0
    if prec == "fp64":
        out = to_np(hub.apply_M(to_dev(phi), torch.ones((w.Nt, w.V), dtype=torch.complex128, device=dev())))
        ref_phi = phi
    else:
        p32 = phi.astype(np.float32)
        out = to_np(hub.apply_M_c64(to_dev(p32), torch.ones((w.Nt, w.V), dtype=torch.complex64, device=dev())))
        ref_phi = p32.astype(np.float64)
    # (M 1)_t = 1 - B_t e^{i phi_{t-1}}  =>  e^{i phi_{t-1}} = B_t (1 - (M 1)_t)
    got = np.roll(B[:, None] * (1.0 - out.astype(np.complex128)), -1, axis=0)
    err = np.abs(got - np.exp(1j * ref_phi))
    if prec == "fp64":
        tol = np.full_like(err, 2e-15)
    else:
        tol = np.where(np.abs(ref_phi) < 6000.0, 2.0 * np.abs(ref_phi) * 2.0 ** -24, 0.0) + 1e-6
    bad = np.argwhere(err > tol)
    assert bad.size == 0, [(float(ref_phi[tuple(i)]), float(err[tuple(i)]), float(tol[tuple(i)])) for i in bad[:5]]


def test_context_manager_releases_the_context():
    """`with Hubbard(...) as hub:` destroys the context on exit; a later call is refused
    (HubError for a NULL context), never run on freed memory."""
    from paper_2210_06874_amd import Hubbard, HubError
    w = TINY
    phi, v = draw_inputs(w)
    P, V = to_dev(phi), to_dev(v)
    with Hubbard(w.L, w.Nt, w.beta, w.kappa) as hub:
        ref = hub.apply_M(P, V)
    assert hub._h is None
    with pytest.raises(HubError):
        hub.apply_M(P, V)
    assert torch.isfinite(ref.real).all()


@pytest.mark.parametrize("L,Nt,nrhs,path,delta", [
    (51, 255, 1, "auto", 0.0625), (51, 127, 2, "auto", 0.0625), (51, 60, 4, "auto", 0.0625),
    (51, 1, 1, "auto", 0.0625), (51, 3, 3, "auto", 0.0625), (51, 255, 1, "fused", 0.0625),
    (51, 127, 2, "fused", 0.0625), (51, 60, 4, "fused", 0.0625), (51, 1, 1, "fused", 0.0625),
    (51, 3, 3, "fused", 0.0625), (102, 5, 3, "auto", 0.0625), (102, 1, 2, "auto", 0.0625),
    (102, 3, 2, "auto", 0.08), (102, 2, 1, "auto", 0.1)])
def test_production_lengths_at_odd_shapes(L, Nt, nrhs, path, delta):
    """The compile-time L = 51 and L = 102 kernels on both sides of the two-workgroup switch
    (fewer than 256 slices), with several right-hand sides, a single slice and odd N_t: M, M^dag,
    FP32 M and M^dag and the force on sampled slices against the oracle's Krylov route (at
    L = 51 FP32 both the polynomial-stencil kernel of the default path and the transform kernels).
    At L = 102 the step delta = 1/16 runs both polynomial stencils; 0.08 (3 delta kappa = 0.24) keeps
    the FP32 one and sends FP64 to the split path; 0.1 sends FP32 to the sublattice kernel too."""
    from paper_2210_06874_amd import Hubbard
    print(f"[case] production length L={L} Nt={Nt} nrhs={nrhs} path={path} delta={delta}", flush=True)
    w = Lattice(f"L{L}_Nt{Nt}", L, Nt, delta * Nt, 3.9, nrhs=nrhs)
    phi, v = draw_inputs(w, seed=L + Nt, nrhs=nrhs)
    op = oracle_op(w, mode="expm")
    hub = Hubbard(L, Nt, w.beta, w.kappa, nrhs_max=nrhs, path=path)
    P, V = to_dev(phi), to_dev(v)
    M64, D64 = to_np(hub.apply_M(P, V)), to_np(hub.apply_Mdag(P, V))
    p32, v32 = phi.astype(np.float32), v.astype(np.complex64)
    M32 = to_np(hub.apply_M_c64(to_dev(p32), to_dev(v32)))
    D32 = to_np(hub.apply_Mdag_c64(to_dev(p32), to_dev(v32)))
    g = to_np(hub.force(P, V))
    p64, v64 = p32.astype(np.float64), v32.astype(np.complex128)
    for t in sorted({0, Nt // 2, Nt - 1}):
        tp, tn = (t - 1) % Nt, (t + 1) % Nt
        Bt, Btn = (-1.0 if t == 0 else 1.0), (-1.0 if tn == 0 else 1.0)
        wv = op.apply_E(v[:, tn])
        assert_close_elementwise(M64[:, t], v[:, t] - Bt * op.apply_E(np.exp(1j * phi[tp])[None] * v[:, tp]),
                                 RTOL64, f"M slice {t}")
        assert_close_elementwise(D64[:, t], v[:, t] - Btn * np.exp(-1j * phi[t])[None] * wv, RTOL64, f"Mdag slice {t}")
        assert_close_elementwise(M32[:, t], v64[:, t] - Bt * op.apply_E(np.exp(1j * p64[tp])[None] * v64[:, tp]),
                                 RTOL32, f"M32 slice {t}")
        assert_close_elementwise(D32[:, t], v64[:, t] - Btn * np.exp(-1j * p64[t])[None] * op.apply_E(v64[:, tn]),
                                 RTOL32, f"Mdag32 slice {t}")
        gref = (-2.0 * Btn * (np.exp(1j * phi[t])[None] * v[:, t] * np.conj(wv)).imag).sum(axis=0)
        assert_close_elementwise(g[t], gref, 1e-11, f"force slice {t}")


@pytest.mark.parametrize("beta,Nt,kappa,mu", [(8.0, 128, 1.0, 0.0), (8.0, 128, -1.0, 0.3), (8.0, 96, 1.0, -0.4),
                                             (8.0, 32, 1.0, 0.0), (2.0, 4, -1.0, 0.2)])
def test_polynomial_stencil_and_transform_kernels_at_L51(beta, Nt, kappa, mu):
    """FP32 at L = 51: the default path applies E by a degree-5 polynomial of dk K (the
    truncated Chebyshev series of e^z on the spectrum [-x, x], x = 3|dk|) while x <= 0.25 (here
    x = 0.1875 with either sign of kappa, 0.25 exactly at Nt = 96, where the polynomial's error
    bound is largest) and by the transforms above it (x = 0.75, 1.5), and the forced fused path
    always by the transforms.  Every entry of M and M^dag of both, with mu != 0 (e^{delta mu}
    scales E), within 1e-6 of the largest entry of the oracle's result on the same FP32-rounded
    inputs: FP32 rounding (random shapes show at most 3e-7), so the polynomial's error (at most
    1.1e-8) is invisible and a wrong choice of kernel (x = 0.75 by the polynomial: about 2e-5)
    is not."""
    from paper_2210_06874_amd import Hubbard
    L = 51
    print(f"[case] polynomial vs transform L={L} Nt={Nt} beta={beta} kappa={kappa} mu={mu}", flush=True)
    w = Lattice(f"L{L}_Nt{Nt}", L, Nt, beta, 3.85, kappa=kappa)
    phi, v = draw_inputs(w, seed=Nt + 5, nrhs=1)
    p32, v32 = phi.astype(np.float32), v.astype(np.complex64)
    p64, v64 = p32.astype(np.float64), v32.astype(np.complex128)
    op = O.HubbardOperator(L, Nt, beta, kappa, mu=mu, mode="expm")
    refM, refD = op.apply_M(p64, v64), op.apply_Mdag(p64, v64)
    for path in ("auto", "fused"):
        hub = Hubbard(L, Nt, beta, kappa, path=path, mu=mu)
        P, V = to_dev(p32), to_dev(v32)
        eM = assert_close_elementwise(to_np(hub.apply_M_c64(P, V)), refM, 1e-6, f"M32 {path}")
        eD = assert_close_elementwise(to_np(hub.apply_Mdag_c64(P, V)), refD, 1e-6, f"Mdag32 {path}")
        print(f"    {path}: M {eM:.2e} Mdag {eD:.2e}", flush=True)
