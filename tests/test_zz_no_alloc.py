"""GPU test of hub_force_noalloc (the force entry point that allocates nothing): through the C ABI
it must give hub_force's result, on two calls in a row (the second with fewer right-hand sides
and then a smaller lattice), and refuse sizes beyond its static scratch."""

import numpy as np
import pytest
import torch

import oracle as O
from workloads import PREC, SMALL, STRESS, draw_inputs
from gpu_common import dev, to_dev, to_np, oracle_op, assert_close_elementwise

pytestmark = pytest.mark.gpu


def test_force_noalloc_matches_force_on_successive_calls():
    from paper_2210_06874_amd import Hubbard
    dev()
    hub = Hubbard(PREC.L, PREC.Nt, PREC.beta, PREC.kappa, nrhs_max=4)
    small = Hubbard(SMALL.L, SMALL.Nt, SMALL.beta, SMALL.kappa, nrhs_max=3)
    for w, h, nrhs, seed in [(PREC, hub, 4, 31), (PREC, hub, 2, 32), (SMALL, small, 3, 33)]:
        print(f"[case] force_noalloc {w.name} nrhs={nrhs}", flush=True)
        phi, x = draw_inputs(w, seed=seed, nrhs=nrhs)
        P, X = to_dev(phi), to_dev(x)
        ref = h.force(P, X)
        out = torch.full_like(ref, float("nan"))
        got = h.force_noalloc(P, X, out)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        assert torch.equal(got, ref), f"{w.name} nrhs={nrhs}: differs from hub_force"
        if w is SMALL:
            assert_close_elementwise(to_np(got), O.force(oracle_op(w), phi, x), 1e-12, "force vs oracle")


def test_force_noalloc_refuses_sizes_beyond_its_scratch():
    from paper_2210_06874_amd import Hubbard, HubError
    w = STRESS                              # N = 3,995,136: three right-hand sides exceed 2^23 doubles
    dev()
    hub = Hubbard(w.L, w.Nt, w.beta, w.kappa, nrhs_max=3)
    P = torch.zeros((w.Nt, w.V), dtype=torch.float64, device=dev())
    X = torch.zeros((3, w.Nt, w.V), dtype=torch.complex128, device=dev())
    g = torch.empty_like(P)
    with pytest.raises(HubError, match="HUB_ERR_ARG"):
        hub.force_noalloc(P, X, g)
    X2 = X[:2].contiguous()                 # two fit: same as hub_force
    assert torch.equal(hub.force_noalloc(P, X2, g), hub.force(P, X2))
