"""CPU checks of the C ABI and of the host-side logic (no device calls)."""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest
import scipy.linalg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hub.h")
CSRC = os.path.join(ROOT, "paper_2210_06874_amd", "csrc")


def _lib():
    from paper_2210_06874_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libhubhip.so not built (run __graft_entry__.build())")
    return L, L.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hub_[A-Za-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    L, lib = _lib()
    names = declared_functions()
    assert {"hub_apply_M", "hub_apply_Mdag", "hub_cg_solve", "hub_force"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (hub_\w+)", out))
    assert set(names) <= exported, set(names) - exported
    assert set(names) == set(L.SIGNATURES), "binding and header disagree"


def test_probe_library_exports_its_entry_points():
    """The measurement probe (one DFT row pass by the FFT stages and as an FP32 MFMA GEMM) is
    a library of its own, outside the C ABI, with the matrix cores' own rate beside them: it
    loads and exports exactly its three entry points, and the ABI library exports none of them."""
    L, _ = _lib()
    from paper_2210_06874_amd import build as B
    if not os.path.exists(B.PROBE_LIB):
        pytest.skip("libhubprobe.so not built (run __graft_entry__.build())")
    ctypes.CDLL(B.PROBE_LIB)
    nm = lambda f: set(re.findall(r"\bT (probe_\w+)", subprocess.run(
        ["nm", "-D", "--defined-only", f], capture_output=True, text=True).stdout))
    assert nm(B.PROBE_LIB) == {"probe_dft_rows_fft51", "probe_dft_rows_mfma51", "probe_mfma_peak"}
    assert nm(L.LIB_PATH) == set()


def test_struct_layouts_match_the_binding(tmp_path):
    L, _ = _lib()
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "host", "layout_driver.c"), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines()
    got = {ln.split()[0]: list(map(int, ln.split()[1:])) for ln in lines}
    for cname, cls in (("hub_params", L.HubParams), ("hub_cg_opts", L.HubCgOpts), ("hub_cg_info", L.HubCgInfo),
                       ("hub_traj_opts", L.HubTrajOpts), ("hub_traj_info", L.HubTrajInfo)):
        ref = [ctypes.sizeof(cls)] + [getattr(cls, f[0]).offset for f in cls._fields_]
        assert got[cname] == ref, (cname, got[cname], ref)


def test_argument_errors_before_any_device_call():
    L, lib = _lib()
    h = ctypes.c_void_p()
    assert lib.hub_create(None, None, ctypes.byref(h)) == L.HUB_ERR_ARG
    assert b"NULL" in lib.hub_last_error()
    for bad in [dict(L=0), dict(L=19), dict(L=2048), dict(Nt=0), dict(nrhs_max=0), dict(path=7),
                dict(beta=float("nan")), dict(mu=float("inf")), dict(form=2), dict(form=-1),
                dict(form=1, mu=0.5), dict(form=1, L=1025),
                dict(Nt=2**30, nrhs_max=4), dict(form=1, Nt=2**30, nrhs_max=4)]:   # launch grid
        prm = dict(L=3, Nt=8, beta=2.0, kappa=1.0, nrhs_max=1, path=0, mu=0.0, form=0)
        prm.update(bad)
        p = L.HubParams(prm["L"], prm["Nt"], prm["beta"], prm["kappa"], prm["nrhs_max"], prm["path"], prm["mu"],
                        prm["form"])
        assert lib.hub_create(ctypes.byref(p), None, ctypes.byref(h)) == L.HUB_ERR_ARG, bad
        assert h.value is None
    assert lib.hub_create(ctypes.byref(L.HubParams(3, 8, 2.0, 1.0, 1, 0, 0.0)), None, None) == L.HUB_ERR_ARG
    x = ctypes.c_void_p(1)
    assert lib.hub_apply_M(None, x, x, x, 1, None) == L.HUB_ERR_ARG
    assert lib.hub_apply_Mdag(None, x, x, x, 1, None) == L.HUB_ERR_ARG
    assert lib.hub_force(None, x, x, x, 1, None) == L.HUB_ERR_ARG
    assert lib.hub_action(None, x, x, 1, x, None) == L.HUB_ERR_ARG
    opts = L.HubCgOpts(1e-10, 100, 50, 0, 0)
    assert lib.hub_cg_solve(None, x, x, x, 1, ctypes.byref(opts), None, None) == L.HUB_ERR_ARG
    assert lib.hub_query(None, None, None) == L.HUB_ERR_ARG
    topts = L.HubTrajOpts(3.0, 0.1, 4, 0, opts)
    assert lib.hub_trajectory(None, x, x, x, 1, 0.5, ctypes.byref(topts), None, None) == L.HUB_ERR_ARG
    lib.hub_destroy(None)   # no-op


# ----------------------------------------------------------------------------- host tables
def _tables(tmp_path, L, dk, dmu=0.0):
    exe = tmp_path / "tables"
    if not exe.exists():
        subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, os.path.join(ROOT, "tests", "host", "tables_driver.cpp"),
                        os.path.join(CSRC, "hub_tables.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe), str(L), repr(dk), repr(dmu)], capture_output=True, text=True,
                         check=True).stdout
    lines = out.splitlines()
    if lines[0] == "noplan":
        return None
    plan = list(map(int, lines[0].split()[1:]))[1:]
    pos = list(map(int, lines[1].split()[1:]))
    roots = np.array([[float(a) for a in ln.split()[1:]] for ln in lines if ln.startswith("root")])
    etab = np.array([[float(a) for a in ln.split()[1:]] for ln in lines if ln.startswith("e ")])
    return plan, pos, roots[:, 0] + 1j * roots[:, 1], etab


def _dif(x, plan):
    """In-place decimation-in-frequency stages with the plan's radices (reference model)."""
    L = len(x)
    x = x.astype(complex).copy()
    w = np.exp(-2j * np.pi * np.arange(L) / L)
    Lq = L
    for r in plan:
        m = Lq // r
        for blk in range(L // Lq):
            for n in range(m):
                idx = blk * Lq + n + m * np.arange(r)
                y = np.exp(-2j * np.pi * np.outer(np.arange(r), np.arange(r)) / r) @ x[idx]
                x[idx] = y * w[(n * np.arange(r) * (L // Lq)) % L]
        Lq = m
    return x


@pytest.mark.parametrize("L", [1, 2, 3, 4, 12, 24, 51, 102, 7 * 5, 17])
def test_plan_positions_follow_the_transform(tmp_path, L):
    """The digit-reversed position table is where the in-place transform leaves each
    frequency (checked against numpy's FFT)."""
    plan, pos, roots, _ = _tables(tmp_path, L, 0.1)
    assert int(np.prod(plan)) == L and set(plan) <= {2, 3, 4, 5, 7, 11, 13, 17}
    assert sorted(pos) == list(range(L))
    x = np.random.default_rng(L).normal(size=L) + 1j * np.random.default_rng(L + 1).normal(size=L)
    y = _dif(x, plan)
    np.testing.assert_allclose(y[pos], np.fft.fft(x), atol=1e-9 * np.abs(x).sum())
    np.testing.assert_allclose(roots, np.exp(-2j * np.pi * np.arange(L) / L), atol=2e-16)


@pytest.mark.parametrize("L,dk,dmu", [(3, 0.25, 0.0), (12, 0.125, 0.0), (51, 0.0625, 0.0), (6, 1.5, 0.0),
                                      (6, 0.25, 0.1), (12, 0.125, -0.05), (6, -0.25, 0.0), (6, -1.0, 0.0),
                                      (51, -0.0625, 0.1), (3, -1e-6, 0.0)])
def test_momentum_hopping_table_is_the_2x2_exponential(tmp_path, L, dk, dmu):
    """E(k)/L^2 at every transform position equals scipy's expm of dk [[0, f], [conj f, 0]] + dmu,
    for either sign of dk (a negative kappa or beta gives the hole operator M[-phi, -kappa])."""
    plan, pos, _, etab = _tables(tmp_path, L, dk, dmu)
    inv = np.empty(L, dtype=int)
    inv[pos] = np.arange(L)
    for p1 in range(L):
        for p2 in range(L):
            k1, k2 = 2 * np.pi * inv[p1] / L, 2 * np.pi * inv[p2] / L
            f = 1 + np.exp(-1j * k1) + np.exp(-1j * k2)
            E = scipy.linalg.expm(dk * np.array([[0, f], [np.conj(f), 0]]) + dmu * np.eye(2))
            c, sr, si = etab[p1 * L + p2] * L * L
            tol = 5e-15 * max(1.0, np.abs(E).max())      # a few ulp of the largest entry
            np.testing.assert_allclose([c, sr + 1j * si], [E[0, 0].real, E[0, 1]], rtol=0, atol=tol)
            np.testing.assert_allclose(E[1, 0], sr - 1j * si, rtol=0, atol=tol)


def _poly(tmp_path, x, deg):
    _tables(tmp_path, 3, 0.1)                         # builds the driver
    out = subprocess.run([str(tmp_path / "tables"), "poly", repr(x), str(deg)], capture_output=True, text=True,
                         check=True).stdout.splitlines()
    err = float(out[0].split()[1])
    a0 = float(out[1].split()[1])
    ratios = [float(v) for v in out[2].split()[1:]]
    return err, np.concatenate([[a0], a0 * np.cumprod(ratios)])


@pytest.mark.parametrize("x,deg", [(0.0, 5), (5e-4, 5), (0.05, 5), (0.1875, 5), (0.25, 5), (0.5, 5),
                                   (0.1875, 9), (0.25, 9), (0.25, 10)])
def test_exp_polynomial_of_the_stencil(tmp_path, x, deg):
    """The polynomial p with which the stencil applies exp(dk K), on the spectrum [-x, x] of dk K
    (x = 3|dk|): degree 5 (FP32) and 9 (FP64).  Rebuilt from a_0 and the ratios the kernel uses,
    it is the Chebyshev series of e^z on [-x, x] truncated at its degree (coefficients 2 I_j(x),
    here from scipy's modified Bessel functions; the Taylor polynomial below x = 1e-3), its
    reported error is max |p(z) - e^z| on a dense grid (in long double), and that error obeys the
    truncation bound 2 (x/2)^{d+1} e^x / (d+1)!: 1.1e-8 at the largest FP32 step x = 0.25, 1.9e-9
    at the paper's x = 0.1875; 2.9e-17 in degree 9 there (6e-17 with the coefficients rounded to
    double, as the device uses them), below FP64 rounding."""
    import scipy.special
    err, a = _poly(tmp_path, x, deg)
    if x < 1e-3:
        ref = 1.0 / np.array([math.factorial(k) for k in range(deg + 1)])
    else:
        c = np.array([scipy.special.iv(j, x) * (1.0 if j == 0 else 2.0) for j in range(deg + 1)])
        ref = np.polynomial.chebyshev.cheb2poly(c) / x ** np.arange(deg + 1)
    z = np.linspace(-x, x, 20001)
    np.testing.assert_allclose(np.polynomial.polynomial.polyval(z, a), np.polynomial.polynomial.polyval(z, ref),
                               rtol=0, atol=1e-15)
    zl = z.astype(np.longdouble)
    p = np.zeros_like(zl)
    for ak in a.astype(np.longdouble)[::-1]:
        p = p * zl + ak
    # the coefficients here are the library's long-double ones rounded to double and rebuilt as
    # a_0 times a product of ratios (the device takes the ratios): each a_k is within a few
    # units of 2^-53 of the library's, so the polynomial moves by at most 4 2^-53 e^x
    dense = float(np.abs(p - np.exp(zl)).max())
    rnd = 4 * 2.0 ** -53 * math.exp(x)
    assert abs(dense - err) <= rnd, (err, dense)
    bound = 2 * (x / 2) ** (deg + 1) * math.exp(x) / math.factorial(deg + 1)
    assert err <= bound + 1e-18 and dense <= bound + rnd, (err, dense, bound)
    if deg == 5 and x <= 0.25:
        assert err <= 1.2e-8
    if deg == 9 and x <= 0.1875:
        assert err <= 1.1e-16 and dense <= 1.1e-16


def test_unsupported_lengths_have_no_plan(tmp_path):
    assert _tables(tmp_path, 19, 0.1) is None
    assert _tables(tmp_path, 23 * 2, 0.1) is None


def test_plain_c_client_compiles_and_links(tmp_path):
    """The C ABI is usable from C alone: the client in tests/host/abi_driver.c builds with
    gcc against include/hub.h and the library, and starts (usage message without args)."""
    exe = tmp_path / "abi_driver"
    subprocess.run(["gcc", "-std=c99", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host", "abi_driver.c"),
                    "-L", os.path.join(ROOT, "paper_2210_06874_amd"), "-lhubhip", "-L/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath," + os.path.join(ROOT, "paper_2210_06874_amd"), "-Wl,-rpath,/opt/rocm/lib",
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 1 and "usage" in r.stderr


def test_host_tables_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The host-side table builder (plans, roots, E(k)) built with AddressSanitizer and
    UBSan (fatal on the first report) runs clean for every supported kind of length and
    prints exactly what the plain build prints."""
    src = [os.path.join(ROOT, "tests", "host", "tables_driver.cpp"), os.path.join(CSRC, "hub_tables.cpp")]
    plain, san = tmp_path / "tables_plain", tmp_path / "tables_san"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, *src, "-o", str(plain)], check=True)
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-I", CSRC, *src, "-o", str(san)], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    for L, dk, dmu in [(1, 0.1, 0.0), (2, 0.3, 0.0), (3, 0.1, 0.2), (17, 0.05, 0.0), (51, 0.0625, -0.1),
                       (102, 0.0625, 0.0), (19, 0.1, 0.0), (6, -1.0, 0.0), (51, -0.0625, 0.0)]:
        a = subprocess.run([str(plain), str(L), repr(dk), repr(dmu)], capture_output=True, text=True, check=True)
        b = subprocess.run([str(san), str(L), repr(dk), repr(dmu)], capture_output=True, text=True, env=env)
        assert b.returncode == 0, (L, b.stderr[-2000:])
        assert "runtime error" not in b.stderr and "AddressSanitizer" not in b.stderr, (L, b.stderr[-2000:])
        assert a.stdout == b.stdout, L


def test_binding_rejects_an_initial_guess_with_another_rhs_count():
    """cg_solve hands the library x's pointer alone, sized for chi's right-hand sides: an x0
    with fewer (or more) right-hand sides than chi is refused before any library call.
    Checked on the CPU with a binding object that has no library context behind it."""
    import torch
    from paper_2210_06874_amd import Hubbard

    class NoLib:
        def __getattr__(self, name):
            raise AssertionError(f"library call {name} reached")

    hub = Hubbard.__new__(Hubbard)
    hub.device, hub.lib, hub._h = torch.device("cpu"), NoLib(), None
    hub.L, hub.Nt, hub.V = 2, 3, 8
    phi = torch.zeros((3, 8), dtype=torch.float64)
    chi = torch.zeros((2, 3, 8), dtype=torch.complex128)
    for n0 in (1, 3):
        with pytest.raises(ValueError, match="right-hand sides"):
            hub.cg_solve(phi, chi, x0=torch.zeros((n0, 3, 8), dtype=torch.complex128))
    with pytest.raises(ValueError, match="right-hand sides"):
        hub.cg_solve(phi, chi, x0=torch.zeros((3, 8), dtype=torch.complex128))
