"""Hybrid Monte Carlo trajectories of the Hubbard field on the device (Sec. 2).

Each trajectory: heat bath chi = M rho (rho ~ e^{-rho^dag rho}), momenta pi ~ e^{-pi^2/2},
molecular dynamics of H = pi^2/2 + phi^2/(2 delta U) + chi^dag (M M^dag)^{-1} chi with the
adjoint force, and acceptance with probability min(1, e^{-dH}).  The integrator is the
leapfrog or the second-order minimum-norm scheme of Omelyan, Mryglod and Folk (two force
evaluations per step, the last momentum update of a step merged with the first of the next).
The whole trajectory runs in the library (hub_trajectory): the random numbers are inputs,
every array operation is a library kernel, and the FP64 accept/reject decision is taken on
the two device-reduced energies.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch


@dataclass
class Trajectory:
    accepted: bool
    dH: float
    H0: float
    H1: float
    cg_iters: int
    n_forces: int


def trajectory(hub, phi: torch.Tensor, U: float, pi0: torch.Tensor, rho: torch.Tensor, u: float,
               n_md: int, eps: float, tol: float = 1e-10, prec: str = "mixed",
               max_iter: int = 200000, integrator: str = "leapfrog") -> Trajectory:
    """One HMC trajectory; `phi` (float64 [Nt, V] on the device) is updated in place and
    restored when the trajectory is rejected.  integrator: "leapfrog" (n_md + 1 force
    evaluations) or "omelyan" (2 n_md + 1)."""
    if integrator not in ("leapfrog", "omelyan"):
        raise ValueError(f"unknown integrator {integrator!r}")
    info = hub.trajectory(phi, pi0, rho, u, U, n_md, eps, integrator=integrator, tol=tol, prec=prec,
                          max_iter=max_iter)
    return Trajectory(bool(info.accepted), info.dH, info.H0, info.H1, info.cg_iters, info.n_forces)


# ----------------------------------------------------------------------------- Markov chains
@dataclass
class ChainState:
    k: int                 # trajectories done
    accepted: int          # of which accepted
    dH: list               # dH of every trajectory done in this run (nan for a failed one)
    failed: int = 0        # of which ended in a solver failure and counted as rejected


def draw_trajectory_randoms(rng, Nt: int, V: int, nrhs: int = 1):
    """The random numbers of one trajectory, on the host, in this order: momenta
    pi ~ e^{-pi^2/2} (float64 [Nt, V]), heat-bath vectors rho ~ e^{-rho^dag rho}
    (complex128 [nrhs, Nt, V]: real parts, then imaginary parts) and the uniform u."""
    import numpy as np
    pi = rng.normal(0.0, 1.0, size=(Nt, V))
    s = math.sqrt(0.5)
    rho = rng.normal(0.0, s, size=(nrhs, Nt, V)) + 1j * rng.normal(0.0, s, size=(nrhs, Nt, V))
    return pi, rho, float(rng.random())


def save_checkpoint(path: str, phi, rng, state: ChainState) -> None:
    """Field, generator state and counters in one .npz (no pickled objects), written to a
    temporary file and renamed, so an interrupted write never replaces a good checkpoint."""
    import json
    import os
    import numpy as np
    phi_h = phi.detach().cpu().numpy() if isinstance(phi, torch.Tensor) else np.asarray(phi)
    tmp = path + ".tmp.npz"
    np.savez(tmp, phi=phi_h, k=np.int64(state.k), accepted=np.int64(state.accepted),
             failed=np.int64(state.failed), rng=np.array(json.dumps(rng.bit_generator.state)))
    os.replace(tmp, path)


def load_checkpoint(path: str):
    """(phi as float64 [Nt, V] numpy, generator, ChainState) from save_checkpoint's file."""
    import json
    import numpy as np
    with np.load(path, allow_pickle=False) as z:
        st = json.loads(str(z["rng"]))
        bg = getattr(np.random, st["bit_generator"])()
        bg.state = st
        failed = int(z["failed"]) if "failed" in z.files else 0
        return np.array(z["phi"]), np.random.Generator(bg), ChainState(int(z["k"]), int(z["accepted"]), [], failed)


def run_chain(hub, phi: torch.Tensor, U: float, n_traj: int, n_md: int, eps: float, rng, nrhs: int = 1,
              state: ChainState | None = None, checkpoint: str | None = None, every: int = 10,
              reject_failed: bool = False, **traj_kw) -> ChainState:
    """Run trajectories until `n_traj` are done in total (counting those in `state`), drawing
    each trajectory's random numbers from the numpy generator `rng`.  `phi` (device) is the
    chain's field, updated in place.  With `checkpoint`, the field, the generator and the
    counters are saved every `every` trajectories and at the end; a chain resumed from
    load_checkpoint continues exactly as if it had not stopped.

    A solve that does not converge or breaks down (the molecular dynamics ran into a nearly
    singular M, close to a zero of det M) raises, unless `reject_failed`: then the trajectory
    counts as rejected (the library has restored phi), its dH is recorded as nan and
    `state.failed` counts it."""
    from ._lib import HubError, HUB_ERR_NOCONV, HUB_ERR_NONFINITE
    state = ChainState(0, 0, []) if state is None else state
    while state.k < n_traj:
        pi, rho, u = draw_trajectory_randoms(rng, hub.Nt, hub.V, nrhs)
        try:
            tr = trajectory(hub, phi, U, torch.from_numpy(pi).to(phi.device),
                            torch.from_numpy(rho).to(phi.device), u, n_md, eps, **traj_kw)
        except HubError as e:
            if not (reject_failed and e.status in (HUB_ERR_NOCONV, HUB_ERR_NONFINITE)):
                raise
            tr = None
        state.k += 1
        if tr is None:
            state.failed += 1
            state.dH.append(math.nan)
        else:
            state.accepted += int(tr.accepted)
            state.dH.append(tr.dH)
        if checkpoint and (state.k % every == 0 or state.k == n_traj):
            save_checkpoint(checkpoint, phi, rng, state)
    return state
