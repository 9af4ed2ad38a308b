"""Shared helpers of the GPU parity tests (inputs come from workloads/, expected values from oracle/)."""
import numpy as np
import pytest
import torch

import oracle as O


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def to_np(t):
    return t.detach().cpu().numpy()


def oracle_op(w, mode=None, L=None, Nt=None, beta=None):
    return O.HubbardOperator(w.L if L is None else L, w.Nt if Nt is None else Nt,
                             w.beta if beta is None else beta, w.kappa, mode=mode)


def assert_close_elementwise(got, ref, rtol, what=""):
    """|got - ref| <= rtol * max|ref| for every element (max-norm relative)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(got - ref).max() / scale
    assert err <= rtol, f"{what}: max elementwise error {err:.3e} > {rtol:.1e}"
    return err
