"""Checkpoints of HMC chains (host side): the field, the generator state and the counters
round-trip through one .npz without pickled objects."""
import numpy as np

from paper_2210_06874_amd import hmc


def test_checkpoint_round_trip(tmp_path):
    rng = np.random.default_rng(123)
    for _ in range(3):
        hmc.draw_trajectory_randoms(rng, 4, 8, 2)
    phi = np.random.default_rng(5).normal(size=(4, 8))
    path = str(tmp_path / "chain.npz")
    hmc.save_checkpoint(path, phi, rng, hmc.ChainState(3, 2, [0.1, -0.2, 0.3], failed=1))
    phi2, rng2, st = hmc.load_checkpoint(path)
    assert np.array_equal(phi2, phi) and st.k == 3 and st.accepted == 2 and st.failed == 1
    a = hmc.draw_trajectory_randoms(rng, 4, 8, 2)
    b = hmc.draw_trajectory_randoms(rng2, 4, 8, 2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    with np.load(path, allow_pickle=False) as z:      # plain arrays only
        assert set(z.files) == {"phi", "k", "accepted", "failed", "rng"}


def test_checkpoint_without_a_failure_count_loads(tmp_path):
    """A checkpoint written before chains counted failed trajectories loads with failed = 0."""
    import json
    rng = np.random.default_rng(9)
    path = str(tmp_path / "old.npz")
    np.savez(path, phi=np.zeros((2, 8)), k=np.int64(4), accepted=np.int64(3),
             rng=np.array(json.dumps(rng.bit_generator.state)))
    _, _, st = hmc.load_checkpoint(path)
    assert (st.k, st.accepted, st.failed) == (4, 3, 0)


def test_randoms_have_the_heat_bath_and_momentum_distributions():
    """<pi^2> = 1, <|rho|^2> = 1 (density e^{-rho^dag rho}), u uniform in [0, 1)."""
    rng = np.random.default_rng(7)
    pis, rhos, us = [], [], []
    for _ in range(200):
        pi, rho, u = hmc.draw_trajectory_randoms(rng, 8, 50, 1)
        pis.append(pi)
        rhos.append(rho)
        us.append(u)
    pis, rhos, us = np.array(pis), np.array(rhos), np.array(us)
    assert abs((pis ** 2).mean() - 1.0) < 0.01
    assert abs((np.abs(rhos) ** 2).mean() - 1.0) < 0.01
    assert abs(rhos.real.var() - 0.5) < 0.01 and abs(rhos.imag.var() - 0.5) < 0.01
    assert us.min() >= 0.0 and us.max() < 1.0 and abs(us.mean() - 0.5) < 0.05
