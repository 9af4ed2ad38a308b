"""Benchmark of the honeycomb Hubbard HMC hot path on one MI355X.

A step is one HMC force evaluation on the L = 51, Nt = 128 lattice (beta = 8,
U = 3.85, kappa = 1): mixed-precision CG solve of (M M^dag) x = chi to a true FP64
residual of 1e-10, the pseudofermion action S = chi^dag x and the adjoint force
dS/dphi.  `value` is the sustained rate of operator applications (M or M^dag, each
counted once; per CG iteration 2, per FP64 residual recomputation 2, the force 1)
over the timed steps.

The input is the field an HMC force sees (Sec. 2): the stored HMC field of this lattice
(workloads/field_L51_Nt128_U3.85_hmc.npz, made by the library's own trajectories from a
cold start; its M M^dag carries the weight det(M M^dag)), with the heat-bath pseudofermion
chi = M rho.  The Gaussian prior draws alone are not solvable at beta = 8 (the CG stalls;
their per-iteration cost is reported by --literal-probe).

Also measured (not part of `value`):
  * the FP64 force step (s per force, FP64 vs mixed);
  * the same force step on the labelled "weak field" (prior draws scaled by delta, iid chi);
  * back-to-back hub_apply_M_c64 / hub_apply_M launches timed with HIP events on
    the launching stream: the roofline of the dominant kernel;
  * the same force step with the linear form of the operator (eq. "ferm_op" as printed,
    a nearest-neighbour stencil) and the roofline of its FP32 apply;
  * the CPU oracle (rank 0, N = 1 only) on a bounded sample of operator applications.

`--stress` replaces all of this by the four-right-hand-side L = 102, Nt = 192 workload
(operator launches for all four vectors, mixed CG iterations); `--copy-floor` by plain
device copies of the same byte counts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--stress] [--copy-floor]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
METRIC = "M-applications/s & s per HMC force, L=51 Nt=128, FP32-mixed vs FP64 @1e-10 res"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_apply_M_c64_L51_Nt128.txt")
TRAFFIC_FILE_LIN = os.path.join(ROOT, "profiles", "traffic_apply_M_c64_linear_L51_Nt128.txt")
TRAFFIC_FILE_TR = os.path.join(ROOT, "profiles", "traffic_apply_M_c64_transform_L51_Nt128.txt")
KERNEL_SOURCES = ["hub_fft.hpp", "hub_kernels.hpp", "hub_math.hpp", "hub_abi.hip", "hub_tables.cpp",
                  "hub_tables.hpp", "hub_internal.hpp"]


def kernel_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2210_06874_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(path: str = TRAFFIC_FILE):
    """HBM bytes per launch of an FP32 operator kernel from the committed rocprofv3
    counter summary, or None when absent or taken on a different kernel source."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_launches(fn, n: int, warm: int = 20) -> float:
    """Average duration (s) of n back-to-back launches, HIP events on the current stream."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(n):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) * 1e-3 / n


def time_graph(fn, per_graph: int = 50, replays: int = 10) -> float:
    """Average duration (s) of one launch of `fn`, captured `per_graph` times in a HIP graph
    and replayed, so host launch overhead is not part of the figure.  HIP events are
    recorded on the stream the graph runs on."""
    import torch
    for _ in range(5):
        fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for _ in range(per_graph):
                fn()
        g.replay()
        s.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        for _ in range(replays):
            g.replay()
        b.record(s)
        b.synchronize()
    return a.elapsed_time(b) * 1e-3 / (per_graph * replays)


def cpu_baseline(w, phi, chi, iters_per_force: int, budget_s: float = 10.0):
    """The CPU oracle as it stands, on the same input as the headline force step: operator
    applications per second on a bounded sample, seconds per CG iteration from a bounded run
    of its textbook CG, and seconds per force = the GPU FP64 solve's iteration count times that
    plus one oracle force.  The dense-E route (E = exp(delta kappa K) from eigh, applied per
    slice by dgemm) with every host core in BLAS; the single-threaded Krylov exp-multiply route
    is reported beside it."""
    import threadpoolctl
    import oracle as O
    ncpu = os.cpu_count() or 1
    with threadpoolctl.threadpool_limits(limits=ncpu, user_api="blas"):
        blas = [dict(api=i["internal_api"], threads=i["num_threads"], version=i.get("version"))
                for i in threadpoolctl.threadpool_info() if i["user_api"] == "blas"]
        t_setup = time.perf_counter()
        op = O.HubbardOperator(w.L, w.Nt, w.beta, w.kappa, mode="dense-E")
        t_setup = time.perf_counter() - t_setup
        op.apply_M(phi, chi)                       # warm-up
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s and n < 400:
            op.apply_M(phi, chi) if n % 2 == 0 else op.apply_Mdag(phi, chi)
            n += 1
        dt = time.perf_counter() - t0
        # the oracle's own CG for a bounded number of iterations (each: M^dag, M, vector updates)
        k = max(4, min(100, int(budget_s / max(1e-3, 2.0 * dt / n))))
        t1 = time.perf_counter()
        O.cg_solve(op, phi, chi, tol=1e-10, max_iter=k)
        t_cg = time.perf_counter() - t1
        x = chi                                    # any vector: the force's cost does not depend on it
        t2 = time.perf_counter()
        O.force(op, phi, x)
        t_force = time.perf_counter() - t2
    # includes the final true-residual check (one more M M^dag) in k iterations' time
    s_it = t_cg / (k + 1)
    t3 = time.perf_counter()
    m = 0
    opk = O.HubbardOperator(w.L, w.Nt, w.beta, w.kappa, mode="expm")
    while time.perf_counter() - t3 < 0.5 * budget_s and m < 100:
        opk.apply_M(phi, chi)
        m += 1
    krylov = m / (time.perf_counter() - t3)
    return {"value": n / dt, "unit": "M-applications/s", "cores": ncpu, "kind": "oracle",
            "s_per_cg_iteration": s_it, "s_per_force": iters_per_force * s_it + t_force,
            "s_per_force_basis": f"{iters_per_force} iterations (the GPU FP64 solve of the same input) "
                                 f"x s per oracle CG iteration + one oracle force ({t_force:.2f} s)",
            "blas": blas, "setup_s_eigh": t_setup,
            "krylov_route_1_thread_M_applications_per_s": krylov,
            "sample": f"{n} alternating M / M^dag applications ({dt:.1f} s) and {k} CG iterations "
                      f"({t_cg:.1f} s) of the FP64 oracle at L={w.L} Nt={w.Nt} on the headline input, "
                      f"dense-E route, BLAS on {ncpu} threads"}


def nrhs_scan(w, dev) -> dict:
    """FP32 application of 1, 2, 4, 8 right-hand sides in one launch (context for the roofline:
    at L = 51 one right-hand side gives 128 slices for 256 compute units)."""
    import torch
    from paper_2210_06874_amd import Hubbard
    from workloads import draw_inputs
    out = {}
    for form in ("exp", "linear"):
        hub = Hubbard(w.L, w.Nt, w.beta, w.kappa, nrhs_max=8, device=dev, form=form)
        rows = {}
        for n in (1, 2, 4, 8):
            phi, chi = draw_inputs(w, nrhs=n)
            p32 = torch.from_numpy(phi).to(dev).float()
            c32 = torch.from_numpy(chi).to(dev).to(torch.complex64)
            o = torch.empty_like(c32)
            t = time_graph(lambda: hub.apply_M_c64(p32, c32, out=o), per_graph=20, replays=5)
            rows[str(n)] = {"us_per_launch": t * 1e6, "us_per_rhs": t * 1e6 / n,
                            "hbm_frac": 20.0 * w.N * n / t / 1e9 / HBM_PEAK_GBS}
        out[form] = rows
    return out


def linear_leg(w, dev, P32, V32, out32, steps: int, warmup: int) -> dict:
    """The force step (on the weak field: the HMC field belongs to the exponential form's
    weight) and the FP32 apply roofline with the linear form of the operator."""
    import torch
    from paper_2210_06874_amd import Hubbard
    from workloads import draw_weak_field
    phi_w, chi_w = draw_weak_field(w)
    P, C = torch.from_numpy(phi_w).to(dev), torch.from_numpy(chi_w).to(dev)
    hub = Hubbard(w.L, w.Nt, w.beta, w.kappa, device=dev, form="linear")
    out = {"input": "weak field (phi = delta * prior draws), chi iid"}
    for prec in ("mixed", "fp64"):
        for _ in range(max(1, warmup)):
            hub.cg_solve(P, C, tol=1e-10, prec=prec, max_iter=200000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        applies = 0
        for _ in range(steps):
            res = hub.cg_solve(P, C, tol=1e-10, prec=prec, max_iter=200000)
            hub.force(P, res.x)
            hub.action(C, res.x)
            applies += 2 * res.iters[0] + 2 * res.reliable_updates[0] + 1
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[prec] = {"s_per_force": dt / steps, "applications_per_s": applies / dt, "cg_iters": res.iters[0],
                     "reliable_updates": res.reliable_updates[0], "true_rel_res": res.true_rel_res[0]}
    t_k = time_graph(lambda: hub.apply_M_c64(P32, V32, out=out32))
    out64 = torch.empty_like(C)
    t_k64 = time_graph(lambda: hub.apply_M(P, C, out=out64))
    alg = 20.0 * w.N
    out["roofline"] = {"bound": "hbm", "achieved": alg / t_k / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": alg / t_k / 1e9 / HBM_PEAK_GBS, "traffic": read_traffic(TRAFFIC_FILE_LIN),
                       "kernel": "hub_apply_M_c64, linear form (k_lin<float, ...>)",
                       "avg_launch_us": t_k * 1e6, "alg_bytes_per_launch": alg,
                       "timing": "HIP graph of 50 launches, events on its stream"}
    out["roofline_apply_M_fp64"] = {"achieved": 2 * alg / t_k64 / 1e9, "frac": 2 * alg / t_k64 / 1e9 / HBM_PEAK_GBS,
                                    "avg_launch_us": t_k64 * 1e6, "alg_bytes_per_launch": 2 * alg}
    return out


def stress_leg(dev, steps: int, persistent: bool = True) -> dict:
    """The four-right-hand-side L = 102, Nt = 192 workload (beta = 12, U = 3.9): one launch
    applies M to all four vectors (FP32 and FP64), and a mixed-precision CG on the weak-field
    input runs `steps` blocks of 50 iterations, all four right-hand sides in every launch: with
    the default kernels (the polynomial stencil), with the sublattice kernel, and (unless
    persistent is False: profilers that cannot follow a cooperative launch) as one persistent
    launch per block of iterations."""
    import torch
    from paper_2210_06874_amd import Hubbard
    from workloads import STRESS, draw_inputs, draw_weak_field
    w = STRESS
    phi, chi = draw_inputs(w, nrhs=w.nrhs)
    P = torch.from_numpy(phi).to(dev)
    C = torch.from_numpy(chi).to(dev)
    P32, C32 = P.float(), C.to(torch.complex64)
    o64, o32 = torch.empty_like(C), torch.empty_like(C32)
    hub = Hubbard(w.L, w.Nt, w.beta, w.kappa, nrhs_max=w.nrhs, device=dev)
    t32 = time_graph(lambda: hub.apply_M_c64(P32, C32, out=o32), per_graph=10, replays=5)
    t64 = time_graph(lambda: hub.apply_M(P, C, out=o64), per_graph=5, replays=4)
    alg32, alg64 = 20.0 * w.N * w.nrhs, 40.0 * w.N * w.nrhs
    pw, cw = draw_weak_field(w, nrhs=w.nrhs)
    Pw, Cw = torch.from_numpy(pw).to(dev), torch.from_numpy(cw).to(dev)
    n_it = 50 * max(1, steps)
    cg = {}
    for mode in (("persistent",) if persistent else ()) + ("sublattice", "two_kernel"):
        hub.set_cg_launch(persistent=(mode == "persistent"), sublattice=(mode == "sublattice"))
        hub.cg_solve(Pw, Cw, tol=1e-10, prec="mixed", max_iter=50, raise_on_error=False)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = hub.cg_solve(Pw, Cw, tol=1e-10, prec="mixed", max_iter=n_it, raise_on_error=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        it = max(res.iters)
        cg[mode] = {"us_per_iteration": dt / it * 1e6, "iterations": it,
                    # 80 B per site-slice on average with the stencil (FP32 angles, x updated every
                    # other iteration), 96 B with a phase table and x every iteration
                    "GBs": (80.0 if mode == "two_kernel" else 96.0) * w.N * w.nrhs * it / dt / 1e9,
                    "persistent_launches": res.persistent_launches}
    hub.set_cg_launch(persistent=False)
    return {"workload": f"{w.name}: L={w.L} Nt={w.Nt} beta={w.beta} U={w.U}, {w.nrhs} right-hand sides per launch",
            "apply_M_c64_us": t32 * 1e6, "apply_M_c64_GBs": alg32 / t32 / 1e9,
            "apply_M_c64_hbm_frac": alg32 / t32 / 1e9 / HBM_PEAK_GBS,
            "apply_M_us": t64 * 1e6, "apply_M_GBs": alg64 / t64 / 1e9,
            "apply_M_hbm_frac": alg64 / t64 / 1e9 / HBM_PEAK_GBS,
            "cg_mixed_us_per_iteration": cg["two_kernel"]["us_per_iteration"],
            "cg_iterations": cg["two_kernel"]["iterations"], "cg_GBs": cg["two_kernel"]["GBs"],
            "cg_mixed_by_launch": cg,
            "timing": "operators: HIP graphs, events on their stream; CG: wall time of one solve of "
                      f"{n_it} iterations (includes its reliable updates); two launches per iteration "
                      "with the default kernels (cg_mixed_us_per_iteration) or the sublattice kernel, "
                      "and one persistent launch per block of iterations"}


def weak_field_leg(w, dev, hub, steps: int) -> dict:
    """The force step on the labelled weak field (prior draws scaled by delta, iid chi): a
    nearly free operator, the stand-in input before an HMC field existed."""
    import torch
    from workloads import draw_weak_field
    phi_w, chi_w = draw_weak_field(w)
    P, C = torch.from_numpy(phi_w).to(dev), torch.from_numpy(chi_w).to(dev)
    out = {"input": "phi = delta * N(0, sqrt(delta U)) prior draws, chi iid"}
    for prec in ("mixed", "fp64"):
        res = hub.cg_solve(P, C, tol=1e-10, prec=prec, max_iter=200000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = hub.cg_solve(P, C, tol=1e-10, prec=prec, max_iter=200000)
            hub.force(P, res.x)
            hub.action(C, res.x)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        out[prec] = {"s_per_force": el, "cg_iters": res.iters[0], "reliable_updates": res.reliable_updates[0],
                     "true_rel_res": res.true_rel_res[0],
                     "applications_per_s": (2 * res.iters[0] + 2 * res.reliable_updates[0] + 1) / el}
    return out


def copy_floor(w, dev) -> dict:
    """The time a plain device-to-device copy (torch's copy kernel, captured in a HIP graph)
    takes to move as many bytes (read + write) as one operator application at L = 51,
    Nt = 128, and at larger sizes: what launch ramp and memory latency leave of the 8 TB/s
    at each size."""
    import torch
    out = {"what": "device-to-device copy, HIP graph of 50 launches, events on its stream",
           "sizes": []}
    cases = [("FP32 application bytes", 20.0 * w.N), ("FP64 application bytes", 40.0 * w.N),
             ("64 MiB", 64.0 * 2 ** 20), ("256 MiB", 256.0 * 2 ** 20), ("1 GiB", 2.0 ** 30)]
    for name, moved in cases:
        n = int(moved // 2) // 4                       # float32 elements read (and written)
        a = torch.full((n,), 1.0, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        t = time_graph(lambda: b.copy_(a), per_graph=50, replays=10)
        out["sizes"].append({"case": name, "bytes_moved": 8.0 * n, "us": t * 1e6,
                             "GBs": 8.0 * n / t / 1e9, "frac_of_hbm_peak": 8.0 * n / t / 1e9 / HBM_PEAK_GBS})
        del a, b
    return out


def dft_pass(w, dev) -> dict:
    """One row pass of the per-slice L-point DFT over every row of every slice of the precision
    workload (2 N_t tiles of L x L complex64, HBM to HBM, one workgroup per tile) in two forms from
    the probe library: the library's own FFT stages on the VALU, and the dense DFT as a real GEMM
    on the FP32 matrix cores.  Each is checked against numpy's FFT, then timed in a HIP graph.
    Decides whether the transform belongs on MFMA."""
    import ctypes

    import numpy as np
    import torch

    from paper_2210_06874_amd import build as B
    if not os.path.exists(B.PROBE_LIB):
        raise RuntimeError(f"{B.PROBE_LIB} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(B.PROBE_LIB)
    for f in (lib.probe_dft_rows_fft51, lib.probe_dft_rows_mfma51):
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
        f.restype = ctypes.c_int
    lib.probe_mfma_peak.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    lib.probe_mfma_peak.restype = ctypes.c_int
    L, ntiles = w.L, 2 * w.Nt
    if L != 51:
        raise ValueError("the probe kernels are compiled for L = 51")
    rng = np.random.default_rng(5)
    x_h = (rng.standard_normal((ntiles, L, L)) + 1j * rng.standard_normal((ntiles, L, L))).astype(np.complex64)
    x = torch.from_numpy(x_h).to(dev)
    y = torch.empty_like(x)
    m = np.arange(L)
    roots = torch.from_numpy(np.exp(-2j * np.pi * m / L).astype(np.complex64)).to(dev)
    th = 2 * np.pi * np.outer(m, m) / L
    G = np.zeros((104, 112))
    G[:L, :L], G[:L, L:2 * L] = np.cos(th), -np.sin(th)
    G[L:2 * L, :L], G[L:2 * L, L:2 * L] = np.sin(th), np.cos(th)
    g = torch.from_numpy(G.astype(np.float32)).to(dev)
    ref = np.fft.fft(x_h.astype(np.complex128), axis=-1)
    scale = np.abs(ref).max()

    def call(f, table):
        rc = f(x.data_ptr(), y.data_ptr(), table.data_ptr(), ntiles,
               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        if rc != 0:
            raise RuntimeError(f"probe launch failed: HIP error {rc}")

    # 51 = 3 * 17, decimation in frequency: position 17 k + j holds frequency k + 3 j
    pos = np.arange(L)
    freq_at = pos // 17 + 3 * (pos % 17)
    moved = 2.0 * ntiles * L * L * 8                         # bytes read + written per pass
    mfma_flops = ntiles * 4 * (104 // 4) * (112 // 16) * 2 * 16 * 16 * 4   # issued per pass
    out = {"what": "one row pass of the 51-point DFT over 2 Nt tiles of 51 x 51 complex64, HBM to HBM, "
                   "HIP graph of 50 launches, events on its stream",
           "bytes_moved": moved}
    for name, f, table, perm in (("fft_valu", lib.probe_dft_rows_fft51, roots, freq_at),
                                 ("dft_mfma_fp32", lib.probe_dft_rows_mfma51, g, pos)):
        y.zero_()
        call(f, table)
        torch.cuda.synchronize()
        err = float(np.abs(y.cpu().numpy() - ref[:, :, perm]).max() / scale)
        if not err < 1e-5:
            raise RuntimeError(f"probe {name}: error {err:.2e} against numpy's FFT")
        t = time_graph(lambda: call(f, table), per_graph=50, replays=10)
        r = {"us": t * 1e6, "GBs": moved / t / 1e9, "max_err_rel": err}
        if name == "dft_mfma_fp32":
            r["mfma_tflops"] = mfma_flops / t / 1e12
            r["mfma_frac_of_fp32_peak"] = mfma_flops / t / 1e12 / 157.3
        out[name] = r
    # the matrix cores' own rate: 1024 workgroups of four waves, each wave 8 * iters independent
    # 16 x 16 x 4 MFMAs on register operands
    nb, iters = 1024, 2048
    rate = {}
    for name, fp64, dt, sheet in (("fp32", 0, torch.float32, 157.3), ("fp64", 1, torch.float64, 78.6)):
        buf = torch.empty(nb * 256, dtype=dt, device=dev)

        def run(buf=buf, fp64=fp64):
            rc = lib.probe_mfma_peak(buf.data_ptr(), nb, iters, fp64,
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
            if rc != 0:
                raise RuntimeError(f"probe launch failed: HIP error {rc}")
        t = time_launches(run, 10, warm=3)
        tf = nb * 4 * iters * 8 * 2048 / t / 1e12
        rate[name] = {"tflops": tf, "datasheet_tflops": sheet, "frac_of_datasheet": tf / sheet}
    out["mfma_rate"] = rate
    out["dft_mfma_fp32"]["mfma_frac_of_measured_rate"] = out["dft_mfma_fp32"]["mfma_tflops"] / rate["fp32"]["tflops"]
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--literal-probe", type=int, default=2000,
                    help="CG iterations to time on the unscaled prior field (0: skip)")
    ap.add_argument("--probe", action="store_true",
                    help="only run 20 FP32 operator launches and a 64 MiB copy (for counter runs)")
    ap.add_argument("--probe-cg", action="store_true",
                    help="only run 60 mixed CG iterations at L = 51, Nt = 128 (one rhs) and at L = 102, "
                         "Nt = 192 (four rhs) on the weak field, and a 64 MiB copy (for counter runs)")
    ap.add_argument("--copy-floor", action="store_true",
                    help="only time plain device-to-device copies (HIP graphs) moving the bytes of one "
                         "FP32 / FP64 operator application and larger sizes, one JSON line")
    ap.add_argument("--probe-dft", action="store_true",
                    help="only check and time one DFT row pass at L = 51, Nt = 128 by the FFT stages "
                         "(VALU) and as an FP32 MFMA GEMM (probe library), one JSON line")
    ap.add_argument("--no-persistent", action="store_true",
                    help="with --stress: leave out the persistent (cooperative) CG launch")
    ap.add_argument("--stress", action="store_true",
                    help="instead of the force step: the four-right-hand-side L = 102, Nt = 192 "
                         "workload (operator launches and mixed CG iterations), one JSON line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU and this benchmark measures one GPU; "
              "--gpus must be 1 (several GPUs would each take independent right-hand sides or a "
              "block of time slices)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2210_06874_amd import Hubbard
    from workloads import PREC, draw_complex, draw_inputs, load_hmc_field

    w = PREC
    dev = torch.device("cuda", 0)
    if args.probe:
        phi, chi = draw_inputs(w)
        hub = Hubbard(w.L, w.Nt, w.beta, w.kappa, device=dev)
        P32 = torch.from_numpy(phi).to(dev).float()
        V32 = torch.from_numpy(chi).to(dev).to(torch.complex64)
        out32 = torch.empty_like(V32)
        hub_lin = Hubbard(w.L, w.Nt, w.beta, w.kappa, device=dev, form="linear")
        hub_tr = Hubbard(w.L, w.Nt, w.beta, w.kappa, device=dev, path="fused")
        for h in (hub, hub_lin, hub_tr):        # polynomial stencil, linear stencil, transforms
            for _ in range(20):
                h.apply_M_c64(P32, V32, out=out32)
        a = torch.full((16 * 1024 * 1024,), 1.0, dtype=torch.float32, device=dev)   # 64 MiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print("probe done")
        return 0
    if args.probe_cg:
        from workloads import STRESS, draw_weak_field
        for wl, n in ((w, 1), (STRESS, STRESS.nrhs)):
            pw, cw = draw_weak_field(wl, nrhs=n)
            hub = Hubbard(wl.L, wl.Nt, wl.beta, wl.kappa, nrhs_max=n, device=dev)
            r = hub.cg_solve(torch.from_numpy(pw).to(dev), torch.from_numpy(cw).to(dev), tol=1e-10,
                             prec="mixed", max_iter=60, raise_on_error=False)
            torch.cuda.synchronize()
            print(f"{wl.name}: {n} rhs, {max(r.iters)} mixed CG iterations", flush=True)
            hub.close()
        a = torch.full((16 * 1024 * 1024,), 1.0, dtype=torch.float32, device=dev)   # 64 MiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print("probe done")
        return 0
    if args.stress:
        print(json.dumps(stress_leg(dev, args.steps, persistent=not args.no_persistent)))
        return 0
    if args.copy_floor:
        print(json.dumps(copy_floor(w, dev)))
        return 0
    if args.probe_dft:
        print(json.dumps(dft_pass(w, dev)))
        return 0
    # the headline input: the stored HMC field, heat-bath chi = M rho (rho seeded)
    phi_h, field_meta = load_hmc_field()
    rho_h = draw_complex(w, seed=11)
    hub = Hubbard(w.L, w.Nt, w.beta, w.kappa, device=dev)
    P = torch.from_numpy(phi_h).to(dev)
    C = hub.apply_M(P, torch.from_numpy(rho_h).to(dev))

    def step(prec, P=P, C=C):
        res = hub.cg_solve(P, C, tol=1e-10, prec=prec, max_iter=200000)
        g = hub.force(P, res.x)
        S = hub.action(C, res.x)
        return res, g, S

    for _ in range(args.warmup):
        step("mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    applies = 0
    last = None
    for _ in range(args.steps):
        res, g, S = step("mixed")
        applies += 2 * res.iters[0] + 2 * res.reliable_updates[0] + 1
        last = res
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3

    # FP64 path for the same force (s per force comparison)
    step("fp64")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n64 = max(1, args.steps // 2)
    for _ in range(n64):
        res64, g64, S64 = step("fp64")
    torch.cuda.synchronize()
    s_force_fp64 = (time.perf_counter() - t1) / n64
    g_mixed = g.cpu().numpy()
    g_fp64 = g64.cpu().numpy()
    force_diff = float(np.linalg.norm(g_mixed - g_fp64) / np.linalg.norm(g_fp64))
    weak = weak_field_leg(w, dev, hub, max(1, args.steps // 2))

    # dominant kernel: the FP32 operator the mixed CG iterates with (same template and launch)
    P32 = P.float()
    V32 = C.to(torch.complex64)
    out32 = torch.empty_like(V32)
    out64 = torch.empty_like(C)
    t_k32 = time_graph(lambda: hub.apply_M_c64(P32, V32, out=out32))
    t_k64 = time_graph(lambda: hub.apply_M(P, C, out=out64))
    t_loop32 = time_launches(lambda: hub.apply_M_c64(P32, V32, out=out32), 300)
    alg32 = 20.0 * w.N          # read v (8N) + phi (4N), write out (8N)
    alg64 = 40.0 * w.N
    traffic = read_traffic(TRAFFIC_FILE)
    # the degree-5 polynomial stencil: per site and sweep, K (two complex adds, 4 flops) and the
    # nested update (one complex scale-add, 4 flops); the phase product (6) and the epilogue (2)
    tay_flops = w.N * (5 * 8.0 + 6.0 + 2.0)
    roof = {"bound": "hbm", "achieved": alg32 / t_k32 / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": alg32 / t_k32 / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "hub_apply_M_c64 (k_exp_poly<float, 51, 512, 5, 2, 1>: degree-5 polynomial of delta kappa K "
                      "as a stencil, two workgroups per slice)",
            "avg_launch_us": t_k32 * 1e6, "avg_launch_us_python_loop": t_loop32 * 1e6,
            "alg_bytes_per_launch": alg32, "site_slices_per_s": w.N / t_k32,
            "alu": {"flops_per_launch": tay_flops, "achieved_tflops": tay_flops / t_k32 / 1e12,
                    "peak_tflops": FP32_VECTOR_PEAK_TFLOPS,
                    "frac": tay_flops / t_k32 / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
                    "convention": "5 sweeps x 8 flops + phase 6 + epilogue 2 per site-slice"},
            "timing": "HIP graph of 50 launches, events on its stream"}
    # the same application by the transform kernels (the forced fused path; every FP64 operator
    # and larger delta kappa use them)
    hub_tr = Hubbard(w.L, w.Nt, w.beta, w.kappa, device=dev, path="fused")
    t_tr = time_graph(lambda: hub_tr.apply_M_c64(P32, V32, out=out32))
    fft_flops = w.Nt * 4 * 5.0 * w.L ** 2 * math.log2(w.L ** 2)
    roof_tr = {"kernel": "k_fused_ct<float, 51, 512, true>: two 2-D transforms forward, the 2 x 2 mix, "
                         "one back per workgroup, two workgroups per slice",
               "avg_launch_us": t_tr * 1e6, "achieved": alg32 / t_tr / 1e9,
               "frac": alg32 / t_tr / 1e9 / HBM_PEAK_GBS,
               "traffic": read_traffic(TRAFFIC_FILE_TR),
               "alu_tflops_5nlog2n": fft_flops / t_tr / 1e12}
    del hub_tr
    roof64 = {"achieved": alg64 / t_k64 / 1e9, "frac": alg64 / t_k64 / 1e9 / HBM_PEAK_GBS,
              "avg_launch_us": t_k64 * 1e6, "alg_bytes_per_launch": alg64}

    lin = linear_leg(w, dev, P32, V32, out32, args.steps, args.warmup)
    batching = nrhs_scan(w, dev)

    # the timed step is almost all CG iterations: two operator kernels that move 80 B per
    # site-slice in FP32 on average (M^dag step: read r, p, the FP32 angle, write t: 28 B;
    # update step: read t, p, r, the angle, write p, r, and every other iteration read and write
    # x for two iterations at once: 44 or 60 B), from the timed region's own clock
    us_it = ms_per_step * 1e3 / last.iters[0]
    cg_iter = {"alg_bytes_per_iteration": 80.0 * w.N, "us_per_iteration": us_it,
               "achieved_GBs": 80.0 * w.N / (us_it * 1e-6) / 1e9,
               "frac_of_hbm_peak": 80.0 * w.N / (us_it * 1e-6) / 1e9 / HBM_PEAK_GBS,
               "note": "wall time of the timed steps over their CG iterations (includes the force, "
                       "action and reliable updates, about 3 %)"}

    probe = None
    if args.literal_probe > 0:
        phi_l, chi_l = draw_inputs(w)
        Pl, Cl = torch.from_numpy(phi_l).to(dev), torch.from_numpy(chi_l).to(dev)
        out = {}
        for prec in ("mixed", "fp64"):
            torch.cuda.synchronize()
            tp = time.perf_counter()
            r = hub.cg_solve(Pl, Cl, tol=1e-10, prec=prec, max_iter=args.literal_probe, raise_on_error=False,
                             history=True)
            torch.cuda.synchronize()
            el = time.perf_counter() - tp
            # true relative residual after each reliable update (every 50 iterations): the
            # non-convergence as it unfolds, not only its end point
            out[prec] = {"iters": r.iters[0], "true_rel_res": r.true_rel_res[0],
                         "us_per_iter": el / max(1, r.iters[0]) * 1e6, "converged": r.converged,
                         "residual_history_every_50": [float(f"{h:.3g}") for h in r.history[0]]}
        probe = out

    line = {
        "metric": METRIC,
        "value": applies / dt,
        "unit": "M-applications/s",
        "value_definition": "applications of the fermion matrix M or M^dag per second (not millions): "
                            "2 per CG iteration, 2 per reliable update and 1 for the force, over the "
                            "timed wall time of the force steps",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"L51_Nt128 HMC field ({field_meta['trajectories']} trajectories from phi = 0 at "
                               f"U = {field_meta['U']}, rms {field_meta['phi_rms']:.3f}), heat-bath chi = M rho; "
                               "one HMC force: mixed CG to 1e-10 + action + force",
                   "L": w.L, "Nt": w.Nt, "beta": w.beta, "U": w.U, "kappa": w.kappa, "nrhs": 1,
                   "parallelism": "single GPU"},
        "cg_iteration": cg_iter,
        "s_per_force_mixed": ms_per_step * 1e-3,
        "s_per_force_fp64": s_force_fp64,
        "cg_iters_mixed": last.iters[0],
        "cg_reliable_updates": last.reliable_updates[0],
        "cg_true_rel_res_mixed": last.true_rel_res[0],
        "cg_iters_fp64": res64.iters[0],
        "force_rel_diff_mixed_vs_fp64": force_diff,
        "weak_field": weak,
        "roofline": roof,
        "roofline_apply_M_fp64": roof64,
        "roofline_apply_M_fp32_transform": roof_tr,
        "linear_form": lin,
        "batching": batching,
        "literal_field_probe": probe,
        "cpu_baseline": None,
    }
    if not args.no_cpu and int(os.environ.get("RANK", "0")) == 0:
        # the oracle's cost per application and per iteration does not depend on the values: it
        # is timed on the same field with rho (a seeded draw) as the vector
        line["cpu_baseline"] = cpu_baseline(w, phi_h, rho_h, res64.iters[0])
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
