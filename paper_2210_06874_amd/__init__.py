"""MI355X (gfx950) hot path of honeycomb Hubbard-model Hybrid Monte Carlo.

A thin Python binding over the C ABI of libhubhip.so (include/hub.h): torch
tensors supply device memory and the current HIP stream; every arithmetic step
runs in the library's HIP kernels.  Names follow the paper (Sec. 2): the
fermion matrix M[phi], the pseudofermion chi, the solution x = (M M^dag)^{-1} chi,
the action S = chi^dag x and its force dS/dphi.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import HubError, HUB_OK

__all__ = ["Hubbard", "CgResult", "HubError", "PseudofermionAction", "reweight"]

_PREC = {"fp64": _lib.HUB_PREC_FP64, "mixed": _lib.HUB_PREC_MIXED}
_PATH = {"auto": _lib.HUB_PATH_AUTO, "fused": _lib.HUB_PATH_FUSED, "split": _lib.HUB_PATH_SPLIT}
_PATH_NAME = {v: k for k, v in _PATH.items()}
_FORM = {"exp": _lib.HUB_FORM_EXP, "linear": _lib.HUB_FORM_LINEAR}
_INTEGRATOR = {"leapfrog": _lib.HUB_MD_LEAPFROG, "omelyan": _lib.HUB_MD_OMELYAN}


def reweight(obs, theta) -> complex:
    """Sec. 3 reweighting of samples drawn with the weight |p|: <O>_p = <O e^{i theta}> / <e^{i theta}>,
    from per-sample observables and phases theta (Hubbard.sign_phase); host-side statistics."""
    import numpy as np
    z = np.exp(1j * np.asarray(theta, dtype=float))
    return complex(np.mean(np.asarray(obs) * z) / np.mean(z))


def _stream_ptr(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class CgResult:
    x: torch.Tensor
    status: int
    iters: list
    reliable_updates: list
    true_rel_res: list
    recursive_rel_res: list
    history: list | None = None     # per rhs: true relative residual after each reliable update
    persistent_launches: int = 0    # persistent CG launches of the solve (0: two per iteration)

    @property
    def converged(self) -> bool:
        return self.status == HUB_OK


class Hubbard:
    """One lattice: L x L honeycomb torus (V = 2 L^2 sites), Nt slices, beta, kappa.

    form="exp" applies the exponential transfer-matrix form of the fermion matrix,
    form="linear" the linear form of eq. "ferm_op" as printed (mu = 0 only).
    """

    def __init__(self, L: int, Nt: int, beta: float, kappa: float = 1.0, nrhs_max: int = 1,
                 path: str = "auto", device=None, mu: float = 0.0, form: str = "exp"):
        self.lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.L, self.Nt, self.beta, self.kappa, self.nrhs_max = L, Nt, float(beta), float(kappa), nrhs_max
        self.mu = float(mu)
        self.form = form
        self.V = 2 * L * L
        self.N = self.V * Nt
        prm = _lib.HubParams(L, Nt, float(beta), float(kappa), nrhs_max, _PATH[path], float(mu), _FORM[form])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self.lib.hub_create(ctypes.byref(prm), _stream_ptr(self.device), ctypes.byref(h)))
        self._h = h
        p, lds = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(self.lib.hub_query(self._h, ctypes.byref(p), ctypes.byref(lds)))
        self.path = _PATH_NAME[p.value]
        self.lds_bytes = lds.value

    def close(self):
        """Release the context's device memory now (also done when the object is collected)."""
        if getattr(self, "_h", None):
            self.lib.hub_destroy(self._h)
            self._h = None

    def __enter__(self) -> "Hubbard":
        return self

    def __exit__(self, *exc) -> None:
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ argument checks
    def _vec(self, v: torch.Tensor, dtype=torch.complex128, name="vector") -> tuple[torch.Tensor, int]:
        if not isinstance(v, torch.Tensor) or v.device != self.device:
            raise ValueError(f"{name} must be a tensor on {self.device}")
        if v.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {v.dtype}")
        if v.dim() == 2:
            v = v.unsqueeze(0)
        if v.dim() != 3 or tuple(v.shape[1:]) != (self.Nt, self.V):
            raise ValueError(f"{name} must have shape [nrhs, {self.Nt}, {self.V}], got {tuple(v.shape)}")
        if not v.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return v, v.shape[0]

    def _phi(self, phi: torch.Tensor, dtype=torch.float64) -> torch.Tensor:
        if not isinstance(phi, torch.Tensor) or phi.device != self.device or phi.dtype != dtype:
            raise ValueError(f"phi must be a {dtype} tensor on {self.device}")
        if tuple(phi.shape) != (self.Nt, self.V) or not phi.is_contiguous():
            raise ValueError(f"phi must be contiguous with shape [{self.Nt}, {self.V}]")
        return phi

    @staticmethod
    def _p(t: torch.Tensor) -> ctypes.c_void_p:
        return ctypes.c_void_p(t.data_ptr())

    # ------------------------------------------------------------------ operators
    def _out(self, out, like: torch.Tensor, name="out") -> torch.Tensor:
        """A caller-supplied output must match what the kernels write exactly: the library
        sees only its pointer, so a short or strided buffer would be overrun."""
        if (not isinstance(out, torch.Tensor) or out.device != like.device or out.dtype != like.dtype
                or tuple(out.shape) != tuple(like.shape) or not out.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {like.dtype} tensor of shape "
                             f"{tuple(like.shape)} on {like.device}")
        return out

    def _apply(self, fn, phi, v, cdtype, rdtype, out=None):
        phi = self._phi(phi, rdtype)
        v3, nrhs = self._vec(v, cdtype)
        o = torch.empty_like(v3) if out is None else self._out(out, v).view(v3.shape)
        with torch.cuda.device(self.device):
            _lib.check(fn(self._h, self._p(phi), self._p(v3), self._p(o), nrhs, _stream_ptr(self.device)))
        return o if v.dim() == 3 else o[0]

    def apply_M(self, phi, v, out=None):
        """M[phi] v in FP64 (complex128 [nrhs, Nt, V] or [Nt, V])."""
        return self._apply(self.lib.hub_apply_M, phi, v, torch.complex128, torch.float64, out)

    def apply_Mdag(self, phi, v, out=None):
        """M[phi]^dag v in FP64."""
        return self._apply(self.lib.hub_apply_Mdag, phi, v, torch.complex128, torch.float64, out)

    def apply_M_c64(self, phi32, v, out=None):
        """M[phi] v in FP32 (complex64 vectors, float32 phi)."""
        return self._apply(self.lib.hub_apply_M_c64, phi32, v, torch.complex64, torch.float32, out)

    def apply_Mdag_c64(self, phi32, v, out=None):
        """M[phi]^dag v in FP32."""
        return self._apply(self.lib.hub_apply_Mdag_c64, phi32, v, torch.complex64, torch.float32, out)

    # ------------------------------------------------------------------ time slabs
    def _slab_args(self, t0, phi, v, halo, cdtype, rdtype, phi_halo=None, name="in"):
        if not isinstance(phi, torch.Tensor) or phi.device != self.device or phi.dtype != rdtype \
                or phi.dim() != 2 or phi.shape[1] != self.V or not phi.is_contiguous():
            raise ValueError(f"phi must be a contiguous {rdtype} tensor [nt, {self.V}] on {self.device}")
        nt = phi.shape[0]
        if not isinstance(v, torch.Tensor) or v.device != self.device or v.dtype != cdtype:
            raise ValueError(f"{name} must be a {cdtype} tensor on {self.device}")
        v3 = v.unsqueeze(0) if v.dim() == 2 else v
        if v3.dim() != 3 or tuple(v3.shape[1:]) != (nt, self.V) or not v3.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape [nrhs, {nt}, {self.V}]")
        nrhs = v3.shape[0]
        if not isinstance(halo, torch.Tensor) or halo.device != self.device or halo.dtype != cdtype \
                or halo.numel() != nrhs * self.V or not halo.is_contiguous():
            raise ValueError(f"the halo must be a contiguous {cdtype} tensor of {nrhs} x {self.V} entries")
        if phi_halo is not None and (not isinstance(phi_halo, torch.Tensor) or phi_halo.device != self.device
                                     or phi_halo.dtype != rdtype or phi_halo.numel() != self.V
                                     or not phi_halo.is_contiguous()):
            raise ValueError(f"phi_halo must be a contiguous {rdtype} tensor of {self.V} entries")
        if not (0 <= int(t0) and int(t0) + nt <= self.Nt):
            raise ValueError(f"slab t0={t0} nt={nt} outside the {self.Nt} slices")
        return nt, v3, nrhs

    def _slab_apply(self, fn, t0, phi, v, halo, cdtype, rdtype, phi_halo=None):
        nt, v3, nrhs = self._slab_args(t0, phi, v, halo, cdtype, rdtype, phi_halo)
        o = torch.empty_like(v3)
        args = [self._h, int(t0), nt, self._p(phi), self._p(v3)]
        if phi_halo is not None:
            args.append(self._p(phi_halo))
        args += [self._p(halo), self._p(o), nrhs, _stream_ptr(self.device)]
        with torch.cuda.device(self.device):
            _lib.check(fn(*args))
        return o if v.dim() == 3 else o[0]

    def apply_M_slab(self, t0, phi, v, phi_halo, v_halo):
        """Rows t0 .. t0+nt-1 of M v from the slab's slices (phi [nt, V], v [nrhs, nt, V]) and
        the halo slice t0-1: phi_halo [V], v_halo [nrhs, V] (FP64)."""
        return self._slab_apply(self.lib.hub_apply_M_slab, t0, phi, v, v_halo, torch.complex128, torch.float64,
                                phi_halo)

    def apply_Mdag_slab(self, t0, phi, v, v_halo):
        """Rows t0 .. t0+nt-1 of M^dag v; v_halo [nrhs, V] is slice t0+nt (mod Nt) (FP64)."""
        return self._slab_apply(self.lib.hub_apply_Mdag_slab, t0, phi, v, v_halo, torch.complex128, torch.float64)

    def apply_M_slab_c64(self, t0, phi32, v, phi_halo, v_halo):
        return self._slab_apply(self.lib.hub_apply_M_slab_c64, t0, phi32, v, v_halo, torch.complex64,
                                torch.float32, phi_halo)

    def apply_Mdag_slab_c64(self, t0, phi32, v, v_halo):
        return self._slab_apply(self.lib.hub_apply_Mdag_slab_c64, t0, phi32, v, v_halo, torch.complex64,
                                torch.float32)

    def force_slab(self, t0, phi, x, x_halo):
        """Rows t0 .. t0+nt-1 of dS/dphi from the slab's solutions x [nrhs, nt, V] and x at slice
        t0+nt (mod Nt), x_halo [nrhs, V]."""
        nt, x3, nrhs = self._slab_args(t0, phi, x, x_halo, torch.complex128, torch.float64, name="x")
        g = torch.empty((nt, self.V), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _lib.check(self.lib.hub_force_slab(self._h, int(t0), nt, self._p(phi), self._p(x3), self._p(x_halo),
                                               self._p(g), nrhs, _stream_ptr(self.device)))
        return g

    # ------------------------------------------------------------------ solver, action, force
    def cg_solve(self, phi, chi, tol: float = 1e-10, max_iter: int = 100000, prec: str = "fp64",
                 reliable_every: int = 50, x0=None, raise_on_error: bool = True,
                 stall_updates: int = 0, history: bool = False) -> CgResult:
        """x = (M M^dag)^{-1} chi by conjugate gradients (true FP64 residual <= tol).

        stall_updates > 0 ends a solve stuck at its attainable accuracy early (HUB_ERR_NOCONV):
        after that many consecutive reliable updates that found the iterated residual below tol
        but no 1 % gain on the best true residual."""
        phi = self._phi(phi)
        chi3, nrhs = self._vec(chi, name="chi")
        if x0 is None:
            x = torch.empty_like(chi3)
            use_x0 = 0
        else:
            # the library reads the guess and writes the solution for nrhs right-hand sides
            # through x's pointer alone, so x0 must hold exactly as many as chi
            x, n0 = self._vec(x0.clone(), name="x0")
            if n0 != nrhs:
                raise ValueError(f"x0 has {n0} right-hand sides, chi has {nrhs}")
            use_x0 = 1
        hist = None
        if history:
            import numpy as np
            hist = np.full((nrhs, int(max_iter) // max(1, int(reliable_every)) + 2), np.nan)
        opts = _lib.HubCgOpts(float(tol), int(max_iter), int(reliable_every), _PREC[prec], use_x0,
                              int(stall_updates), None if hist is None else hist.ctypes.data,
                              0 if hist is None else hist.shape[1])
        info = (_lib.HubCgInfo * nrhs)()
        with torch.cuda.device(self.device):
            st = self.lib.hub_cg_solve(self._h, self._p(phi), self._p(chi3), self._p(x), nrhs,
                                       ctypes.byref(opts), info, _stream_ptr(self.device))
        if raise_on_error:
            _lib.check(st)
        res = CgResult(x if chi.dim() == 3 else x[0], st,
                       [i.iters for i in info], [i.reliable_updates for i in info],
                       [i.true_rel_res for i in info], [i.recursive_rel_res for i in info])
        if hist is not None:
            res.history = [hist[r, :min(info[r].reliable_updates, hist.shape[1])].copy() for r in range(nrhs)]
        res.persistent_launches = info[0].persistent_launches
        return res

    def set_cg_launch(self, persistent: bool = False, barrier_spin_limit: int = 0, sublattice: bool = False) -> None:
        """hub_set_cg_launch: persistent CG launches where they apply (mode 1), two launches per
        iteration of the sublattice kernel the persistent launch is built from (sublattice=True,
        mode 2), or two launches per iteration with the fastest kernels (the default, mode 0);
        barrier_spin_limit > 0 bounds each grid-barrier wait (polls)."""
        mode = 1 if persistent else (2 if sublattice else 0)
        _lib.check(self.lib.hub_set_cg_launch(self._h, mode, int(barrier_spin_limit)))

    def force(self, phi, x, out=None):
        """dS/dphi (float64 [Nt, V]) of S = chi^dag (M M^dag)^{-1} chi from the solutions x."""
        phi = self._phi(phi)
        x3, nrhs = self._vec(x, name="x")
        g = torch.empty((self.Nt, self.V), dtype=torch.float64, device=self.device) if out is None \
            else self._out(out, phi)
        with torch.cuda.device(self.device):
            _lib.check(self.lib.hub_force(self._h, self._p(phi), self._p(x3), self._p(g), nrhs,
                                          _stream_ptr(self.device)))
        return g

    def force_noalloc(self, phi, x, out):
        """hub_force_noalloc: force() into a caller-supplied `out`, with no device allocation
        in the call (the library's static scratch sums the right-hand sides)."""
        phi = self._phi(phi)
        x3, nrhs = self._vec(x, name="x")
        g = self._out(out, phi)
        with torch.cuda.device(self.device):
            _lib.check(self.lib.hub_force_noalloc(self._h, self._p(phi), self._p(x3), self._p(g), nrhs,
                                                  _stream_ptr(self.device)))
        return g

    def action(self, chi, x):
        """S = sum_r Re(chi_r^dag x_r) in FP64, as a 0-dim device tensor."""
        chi3, nrhs = self._vec(chi, name="chi")
        x3, n2 = self._vec(x, name="x")
        if n2 != nrhs:
            raise ValueError("chi and x have different nrhs")
        S = torch.empty((), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _lib.check(self.lib.hub_action(self._h, self._p(chi3), self._p(x3), nrhs, self._p(S),
                                           _stream_ptr(self.device)))
        return S


    # ------------------------------------------------------------------ Sec. 3 weight
    def log_det(self, phi) -> torch.Tensor:
        """(log|det M[phi]|, arg det M[phi]) as a float64 device tensor [2] (hub_log_det)."""
        phi = self._phi(phi)
        out = torch.empty(2, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _lib.check(self.lib.hub_log_det(self._h, self._p(phi), self._p(out), _stream_ptr(self.device)))
        return out

    def sign_phase(self, hole: "Hubbard", phi) -> float:
        """theta of the Sec. 3 weight det(M[phi,mu] M[phi,-mu]^dag) = |p| e^{i theta}: this context
        holds +mu, `hole` the same lattice at -mu; theta = arg det M[phi,mu] - arg det M[phi,-mu],
        reduced to (-pi, pi]."""
        a = self.log_det(phi)[1] - hole.log_det(phi)[1]
        return float(torch.atan2(torch.sin(a), torch.cos(a)))

    # ------------------------------------------------------------------ HMC pieces
    def md_update(self, phi, pi, dSdphi, U: float, eps_pi: float, eps_phi: float):
        """In place: pi -= eps_pi (phi/(delta U) + dSdphi); phi += eps_phi pi."""
        for a in (phi, pi, dSdphi):
            self._phi(a)
        with torch.cuda.device(self.device):
            _lib.check(self.lib.hub_md_update(self._h, self._p(phi), self._p(pi), self._p(dSdphi), float(U),
                                              float(eps_pi), float(eps_phi), _stream_ptr(self.device)))

    def boson_energy(self, phi, pi, U: float):
        """sum pi^2/2 + phi^2/(2 delta U) in FP64, as a 0-dim device tensor."""
        self._phi(phi)
        self._phi(pi)
        E = torch.empty((), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _lib.check(self.lib.hub_boson_energy(self._h, self._p(phi), self._p(pi), float(U), self._p(E),
                                                 _stream_ptr(self.device)))
        return E

    def trajectory(self, phi, pi0, rho, u: float, U: float, n_md: int, eps: float,
                   integrator: str = "leapfrog", tol: float = 1e-10, prec: str = "mixed",
                   max_iter: int = 200000, reliable_every: int = 50) -> "_lib.HubTrajInfo":
        """One HMC trajectory (hub_trajectory): phi is updated in place, or left as it was
        when the trajectory is rejected.  rho: complex128 [nrhs, Nt, V] or [Nt, V]."""
        self._phi(phi)
        self._phi(pi0)
        rho3, nrhs = self._vec(rho, name="rho")
        opts = _lib.HubTrajOpts(float(U), float(eps), int(n_md), _INTEGRATOR[integrator],
                                _lib.HubCgOpts(float(tol), int(max_iter), int(reliable_every), _PREC[prec], 0, 0))
        info = _lib.HubTrajInfo()
        with torch.cuda.device(self.device):
            _lib.check(self.lib.hub_trajectory(self._h, self._p(phi), self._p(pi0), self._p(rho3), nrhs, float(u),
                                               ctypes.byref(opts), ctypes.byref(info), _stream_ptr(self.device)))
        return info


from .autograd import PseudofermionAction  # noqa: E402
