"""GPU parity of hub_log_det, the fermion determinant behind the Sec. 3 weight
det(M[phi,mu] M[phi,-mu]^dag) and its reweighting phase theta, against closed forms and the
oracle's transfer-product determinant."""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import TINY, SMALL, Lattice, draw_inputs, draw_phi
from gpu_common import dev, to_dev, to_np
import closed_forms as CF

pytestmark = pytest.mark.gpu


def _hub(L, Nt, beta, kappa=1.0, mu=0.0, form="exp"):
    from paper_2210_06874_amd import Hubbard
    return Hubbard(L, Nt, beta, kappa, mu=mu, form=form)


def _wrap(a):
    return float(np.angle(np.exp(1j * a)))


@pytest.mark.parametrize("L,Nt,beta,mu", [(3, 8, 2.0, 0.0), (3, 8, 2.0, 0.3), (6, 16, 2.0, -0.7),
                                          (12, 32, 4.0, 0.25), (1, 3, 1.0, 0.5), (24, 16, 2.0, 0.1)])
def test_free_determinant_closed_form(L, Nt, beta, mu):
    """phi = 0: det M = prod_{k,+-} (1 + e^{beta (mu +- kappa |f(k)|)}), real and positive."""
    print(f"[case] log det free L={L} Nt={Nt} beta={beta} mu={mu}", flush=True)
    hub = _hub(L, Nt, beta, mu=mu)
    got = to_np(hub.log_det(torch.zeros((Nt, 2 * L * L), dtype=torch.float64, device=dev())))
    a = np.abs(CF.f_of_k(L)).ravel()
    ref = np.sum(np.log1p(np.exp(beta * (mu + a)))) + np.sum(np.log1p(np.exp(beta * (mu - a))))
    assert abs(got[0] - ref) <= 1e-12 * abs(ref), (got, ref)
    assert abs(got[1]) <= 1e-10          # the arguments of V nearly real pivots, each ~1e-14 off


@pytest.mark.parametrize("mu", [0.0, 0.4])
def test_time_dependent_uniform_field_closed_form(mu):
    """phi_{t,x} = c_t: det M = prod_{k,+-} (1 + e^{i sum c} e^{beta (mu +- kappa |f|)})."""
    L, Nt, beta = 6, 12, 3.0
    c = np.random.default_rng(61).uniform(-1.0, 1.0, size=Nt)
    hub = _hub(L, Nt, beta, mu=mu)
    got = to_np(hub.log_det(to_dev(np.repeat(c[:, None], 2 * L * L, axis=1))))
    a = np.abs(CF.f_of_k(L)).ravel()
    z = np.exp(1j * c.sum())
    terms = np.concatenate([1 + z * np.exp(beta * (mu + a)), 1 + z * np.exp(beta * (mu - a))])
    ref_l, ref_a = np.sum(np.log(np.abs(terms))), _wrap(np.sum(np.angle(terms)))
    assert abs(got[0] - ref_l) <= 1e-12 * abs(ref_l)
    assert abs(_wrap(got[1] - ref_a)) <= 1e-11


@pytest.mark.parametrize("w,mu", [(TINY, 0.0), (TINY, 0.6), (Lattice("L6_Nt16", 6, 16, 2.0, 3.0), -0.3),
                                  (SMALL, 0.0), (SMALL, 0.2)], ids=lambda a: getattr(a, "name", str(a)))
def test_random_field_against_the_oracle(w, mu):
    """Prior draws phi ~ N(0, sqrt(delta U)): log|det M| and arg det M against the oracle's
    dense transfer product."""
    print(f"[case] log det {w.name} mu={mu}", flush=True)
    phi, _ = draw_inputs(w, seed=62)
    hub = _hub(w.L, w.Nt, w.beta, w.kappa, mu=mu)
    got = to_np(hub.log_det(to_dev(phi)))
    ref = O.log_det(O.HubbardOperator(w.L, w.Nt, w.beta, w.kappa, mu=mu), phi)
    assert abs(got[0] - ref[0]) <= 1e-11 * max(1.0, abs(ref[0])), (got, ref)
    assert abs(_wrap(got[1] - ref[1])) <= 1e-9, (got, ref)
    again = to_np(hub.log_det(to_dev(phi)))
    assert np.array_equal(again, got)                       # fixed-order arithmetic


def test_hole_determinant_is_the_conjugate():
    """Sec. 2: on the bipartite lattice det M[-phi, -kappa] = conj det M[phi, kappa], so the
    particle-hole weight is det(M M^dag) >= 0."""
    w = SMALL
    phi, _ = draw_inputs(w, seed=63)
    a = to_np(_hub(w.L, w.Nt, w.beta, 1.0).log_det(to_dev(phi)))
    b = to_np(_hub(w.L, w.Nt, w.beta, -1.0).log_det(to_dev(-phi)))
    assert abs(a[0] - b[0]) <= 1e-11 * abs(a[0]) and abs(_wrap(a[1] + b[1])) <= 1e-9


def test_sign_phase_and_reweighting_against_the_oracle():
    """Sec. 3: theta = arg det M[phi,mu] - arg det M[phi,-mu] on a sample of fields, zero at
    mu = 0, and the reweighted mean <O e^{i theta}> / <e^{i theta}> of an observable (here the
    mean of phi^2 over the lattice) from the device phases against the oracle's."""
    from paper_2210_06874_amd import reweight
    w = TINY
    mu = 0.5
    plus, minus = _hub(w.L, w.Nt, w.beta, mu=mu), _hub(w.L, w.Nt, w.beta, mu=-mu)
    zero = _hub(w.L, w.Nt, w.beta)
    opp = O.HubbardOperator(w.L, w.Nt, w.beta, mu=mu)
    opm = O.HubbardOperator(w.L, w.Nt, w.beta, mu=-mu)
    rng = np.random.default_rng(64)
    th, th_ref, obs = [], [], []
    for _ in range(12):
        phi = draw_phi(w, rng=rng)
        P = to_dev(phi)
        th.append(plus.sign_phase(minus, P))
        th_ref.append(O.sign_phase(opp, opm, phi))
        obs.append(float(np.mean(phi * phi)))
        assert zero.sign_phase(zero, P) == 0.0
    th, th_ref = np.array(th), np.array(th_ref)
    assert np.abs(np.angle(np.exp(1j * (th - th_ref)))).max() <= 1e-9
    assert np.abs(th).max() > 1e-3                           # the sign problem is there
    got, ref = reweight(np.array(obs), th), O.reweight(np.array(obs), th_ref)
    assert abs(got - ref) <= 1e-9 * abs(ref)


def test_log_det_arguments_are_checked():
    from paper_2210_06874_amd import HubError
    big = _hub(25, 2, 1.0)                                   # V = 1250 > 1152
    with pytest.raises(HubError, match="HUB_ERR_ARG"):
        big.log_det(torch.zeros((2, 1250), dtype=torch.float64, device=dev()))
    hot = _hub(3, 8, 12.0)                                   # beta * 3 kappa = 36 > 29
    with pytest.raises(HubError, match="HUB_ERR_ARG"):
        hot.log_det(torch.zeros((8, 18), dtype=torch.float64, device=dev()))
    lin = _hub(3, 8, 2.0, form="linear")
    with pytest.raises(HubError, match="HUB_ERR_ARG"):
        lin.log_det(torch.zeros((8, 18), dtype=torch.float64, device=dev()))
