"""Build libhubhip.so (the C-ABI library) in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhubhip.so")

SOURCES = ["hub_abi.hip", "hub_tables.cpp"]
# a measurement probe kept out of the C ABI (bench.py --probe-dft): its own library
PROBE_SOURCES = ["probe_dft_pass.hip"]
PROBE_LIB = os.path.join(HERE, "libhubprobe.so")
HEADERS = ["hub_internal.hpp", "hub_tables.hpp", "hub_fft.hpp", "hub_kernels.hpp", "hub_math.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall",
    # keep packed FP32 instructions out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, extra_flags=(), out: str | None = None) -> str:
    """Compile every source for gfx950 and link libhubhip.so (or `out`); returns its path.
    The default build also links the probe library libhubprobe.so."""
    lib = LIB if out is None else out
    build_dir = BUILD if out is None else lib + ".objs"
    os.makedirs(build_dir, exist_ok=True)
    srcs = SOURCES + (PROBE_SOURCES if out is None else [])
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(lambda f: _compile(f, build_dir, tuple(extra_flags)), srcs))
    if out is None:
        _link(objs[len(SOURCES):], PROBE_LIB, verbose)
    return _link(objs[:len(SOURCES)], lib, verbose)


def _link(objs, lib: str, verbose: bool) -> str:
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
