"""The C ABI used from plain C (tests/host/abi_driver.c: hipMalloc'd buffers, hub_create,
hub_apply_M, a mixed-precision hub_cg_solve and hub_force, no Python or torch in the
process), checked against the oracle."""
import os
import subprocess

import numpy as np
import pytest

import oracle as O
from workloads import TINY, SMALL, draw_inputs, draw_weak_field
from gpu_common import assert_close_elementwise

pytestmark = pytest.mark.gpu

DRIVER = os.path.join(os.path.dirname(__file__), "host", "abi_driver")


def _run(w, form, phi, chi, tmp_path):
    if not os.path.exists(DRIVER):
        pytest.fail("tests/host/abi_driver is not built: run __graft_entry__.build()")
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as f:
        f.write(np.ascontiguousarray(phi, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(chi, dtype=np.complex128).tobytes())
    r = subprocess.run([DRIVER, str(w.L), str(w.Nt), repr(w.beta), repr(w.kappa), str(form), str(src), str(dst)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = open(dst, "rb").read()
    N = w.N
    vals = np.frombuffer(raw[: 5 * N * 8], dtype=np.float64)
    mv = vals[: 2 * N].view(np.complex128).reshape(w.Nt, w.V)
    x = vals[2 * N: 4 * N].view(np.complex128).reshape(w.Nt, w.V)
    g = vals[4 * N:].reshape(w.Nt, w.V)
    iters = int(np.frombuffer(raw[5 * N * 8: 5 * N * 8 + 4], dtype=np.int32)[0])
    res = float(np.frombuffer(raw[5 * N * 8 + 4:], dtype=np.float64)[0])
    return mv, x, g, iters, res


@pytest.mark.parametrize("form", [0, 1], ids=["exp", "linear"])
def test_c_client_tiny_against_dense_oracle(form, tmp_path):
    w = TINY
    print(f"[case] C client form={form} {w.name}", flush=True)
    phi, chi = draw_inputs(w, seed=31)
    op = (O.HubbardOperator if form == 0 else O.LinearHubbardOperator)(w.L, w.Nt, w.beta, w.kappa)
    mv, x, g, iters, res = _run(w, form, phi, chi[0], tmp_path)
    assert_close_elementwise(mv, op.apply_M(phi, chi)[0], 1e-12, "M chi")
    assert res <= 1e-10 and iters > 0
    x_ref = O.dense_solve_op(op, phi, chi)[0]
    M = op.dense_M(phi)
    cond = np.linalg.cond(M @ M.conj().T)
    assert np.linalg.norm(x - x_ref) <= 2 * cond * 1e-10 * np.linalg.norm(x_ref)
    g_ref = O.force(op, phi, x[None]) if form == 0 else O.force_linear(op, phi, x[None])
    assert_close_elementwise(g, g_ref, 1e-12, "force from the returned x")


def test_c_client_small_weak_field(tmp_path):
    w = SMALL
    phi, chi = draw_weak_field(w, seed=32)
    op = O.HubbardOperator(w.L, w.Nt, w.beta, w.kappa)
    mv, x, g, iters, res = _run(w, 0, phi, chi[0], tmp_path)
    assert_close_elementwise(mv, op.apply_M(phi, chi)[0], 1e-12, "M chi")
    rr = np.linalg.norm(chi[0] - op.apply_A(phi, x[None])[0]) / np.linalg.norm(chi[0])
    assert rr <= 1.01e-10, rr
    assert_close_elementwise(g, O.force(op, phi, x[None]), 1e-12, "force")


def test_c_client_runs_an_hmc_trajectory(tmp_path):
    """hub_trajectory called from plain C: one leapfrog trajectory with rho = chi, against
    the oracle trajectory from the same numbers (decision, dH and the resulting field)."""
    from oracle import hmc as OH
    w = TINY
    phi = draw_weak_field(w, seed=33)[0]
    _, rho = draw_inputs(w, seed=34)
    pi = np.random.default_rng(35).normal(size=(w.Nt, w.V))
    u = 0.5
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as f:
        f.write(np.ascontiguousarray(phi).tobytes())
        f.write(np.ascontiguousarray(rho[0]).tobytes())
        f.write(np.ascontiguousarray(pi).tobytes())
    r = subprocess.run([DRIVER, str(w.L), str(w.Nt), repr(w.beta), repr(w.kappa), "0", str(src), str(dst),
                        repr(w.U), "0.05", "8", repr(u)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = open(dst, "rb").read()
    off = 5 * w.N * 8 + 4 + 8
    accepted = int(np.frombuffer(raw[off: off + 4], dtype=np.int32)[0])
    dH = float(np.frombuffer(raw[off + 4: off + 12], dtype=np.float64)[0])
    phi_after = np.frombuffer(raw[off + 12:], dtype=np.float64).reshape(w.Nt, w.V)
    op = O.HubbardOperator(w.L, w.Nt, w.beta, w.kappa)
    _, _, dH_ref, acc_ref, out_ref = OH.trajectory(op, w.U, phi, pi, rho, u, n_md=8, eps=0.05)
    assert bool(accepted) == acc_ref
    assert abs(dH - dH_ref) <= 1e-7 * max(1.0, abs(dH_ref)), (dH, dH_ref)
    np.testing.assert_allclose(phi_after, out_ref, rtol=0, atol=1e-8)
