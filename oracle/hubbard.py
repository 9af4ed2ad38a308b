"""Plain FP64 CPU oracle for the honeycomb Hubbard-model HMC hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It is deliberately slow and shares no
code with the HIP library: its own geometry, its own exp(delta*kappa*K) (from an
eigen-decomposition or from scipy's Krylov exp-multiply, never a DFT), its own
operators, solver and force.

Paper sections cited below are those of "Stochastic and Tensor Network
simulations of the Hubbard Model" (LATTICE2022):

* Sec. 1, fig. "honeycomb_lattice": two triangular sublattices whose nearest
  neighbours lie on the opposite sublattice (bipartite lattice).
* Sec. 1, particle-hole Hamiltonian: nearest-neighbour hopping -kappa and on-site
  coupling U; the conclusion (Sec. 4) notes that HMC runs use periodic boundaries.
* Sec. 2, eq. "hamiltonian": H = delta/(2U) phi^2 + chi^dag (M M^dag)^{-1} chi + pi^2/2,
  delta = beta/Nt.
* Sec. 2, eq. "ferm_op": the fermion operator couples neighbouring time slices
  through e^{i delta phi} phases and hops between sublattices with strength
  delta*kappa.  HubbardOperator implements the exponential (transfer-matrix) form
  of that operator: slice t couples to slice t-1 through exp(delta*kappa*K) times
  the phase diagonal of slice t-1, with an antiperiodic sign on the wrap.
  LinearHubbardOperator implements the operator exactly as the equation prints it
  (linear in delta*kappa, staggered between the sublattices).
* Sec. 2: chi = M rho with rho ~ e^{-rho^dag rho}; the sampled weight is
  det(M M^dag) e^{-delta phi^2/(2U)}.

Conventions (readings where the paper is silent):
* site index x = s*L^2 + n1*L + n2, s = 0 (A), 1 (B); bonds A(n)-B(n),
  A(n)-B(n-e1), A(n)-B(n-e2) on the L x L torus (multiple bonds add up).
* phase e^{i phi_{t,x}} on every site (phi here is delta times the paper's phi).
* (M v)_t = v_t - B_t * E * D_{t-1} v_{t-1},  B_0 = -1, B_t = +1 otherwise,
  E = exp(delta*kappa*K), D_t = diag(e^{i phi_t}), time indices mod Nt.
* (M^dag v)_t = v_t - B_{t+1} * D_t^* E v_{t+1}.
* away from half filling (Sec. 3) the chemical potential mu multiplies every time hop
  by e^{delta mu}: E = e^{delta mu} exp(delta*kappa*K); the weight is
  det(M[phi,mu] M[phi,-mu]^dag).

Functions carrying no independent pin say "parity unpinned" in their docstring;
all others are pinned by the tests in tests/test_oracle_pins.py (exponential form,
chemical potential), tests/test_oracle_linear.py (linear form: the free determinant, and
at phi != 0 the momentum blocks of a time-dependent uniform field and the determinant
lemma for a field on one site) and tests/test_oracle_hmc.py (trajectories, and the field's
prior variance delta*U without fermions), with planted mistakes in
tests/test_oracle_mutants.py (both forms; the linear-form ones planted consistently in the
dense and matrix-free operators).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = [
    "site_index", "honeycomb_bonds", "hopping_matrix", "hopping_matrix_sparse",
    "hopping_exponential", "antiperiodic_signs", "HubbardOperator", "LinearHubbardOperator",
    "cg_solve", "dense_solve", "action", "force", "force_dense", "force_linear",
    "force_dense_linear", "dense_solve_op", "log_det", "sign_phase", "reweight",
]


# --------------------------------------------------------------------------- geometry
def site_index(L: int, s: int, n1: int, n2: int) -> int:
    """Flat site index of sublattice s (0=A, 1=B) in unit cell (n1, n2), periodic."""
    return s * L * L + (n1 % L) * L + (n2 % L)


def honeycomb_bonds(L: int) -> list[tuple[int, int]]:
    """Nearest-neighbour (A, B) bonds of the L x L honeycomb torus.

    Sec. 1, fig. "honeycomb_lattice": every A site has its three neighbours on the
    B sublattice.  With unit-cell vectors e1, e2 the neighbours of A(n) are
    B(n), B(n - e1), B(n - e2).
    """
    bonds = []
    for n1 in range(L):
        for n2 in range(L):
            a = site_index(L, 0, n1, n2)
            for d1, d2 in ((0, 0), (-1, 0), (0, -1)):
                bonds.append((a, site_index(L, 1, n1 + d1, n2 + d2)))
    return bonds


def hopping_matrix(L: int) -> np.ndarray:
    """Dense real symmetric K with K[x,y] = number of bonds between x and y (Sec. 1)."""
    V = 2 * L * L
    K = np.zeros((V, V))
    for a, b in honeycomb_bonds(L):
        K[a, b] += 1.0
        K[b, a] += 1.0
    return K


def hopping_matrix_sparse(L: int) -> sp.csr_matrix:
    """Sparse copy of hopping_matrix (duplicates summed)."""
    bonds = np.array(honeycomb_bonds(L), dtype=np.int64)
    V = 2 * L * L
    rows = np.concatenate([bonds[:, 0], bonds[:, 1]])
    cols = np.concatenate([bonds[:, 1], bonds[:, 0]])
    data = np.ones(rows.size)
    return sp.csr_matrix((data, (rows, cols)), shape=(V, V))


def hopping_exponential(L: int, delta_kappa: float) -> np.ndarray:
    """E = exp(delta*kappa*K) from the eigen-decomposition of the symmetric K."""
    lam, Q = np.linalg.eigh(hopping_matrix(L))
    return (Q * np.exp(delta_kappa * lam)) @ Q.T


def antiperiodic_signs(Nt: int) -> np.ndarray:
    """B_t: -1 on the wrap block t = 0 (coupling to slice Nt-1), +1 otherwise."""
    B = np.ones(Nt)
    B[0] = -1.0
    return B


# --------------------------------------------------------------------------- operator
class HubbardOperator:
    """The fermion matrix M[phi] in transfer-matrix form (Sec. 2, eq. "ferm_op").

    mode "dense-E": E is the dense V x V matrix exp(delta*kappa*K) (eigh);
    mode "expm":    E v is scipy.sparse.linalg.expm_multiply on the sparse K,
                    usable at every size.
    """

    def __init__(self, L: int, Nt: int, beta: float, kappa: float = 1.0, mode: str | None = None,
                 mu: float = 0.0):
        self.L, self.Nt, self.beta, self.kappa = L, Nt, float(beta), float(kappa)
        self.mu = float(mu)
        self.V = 2 * L * L
        self.N = self.V * Nt
        self.delta = self.beta / Nt
        self.dk = self.delta * self.kappa
        if mode is None:
            mode = "dense-E" if self.V <= 6000 else "expm"
        self.mode = mode
        self.B = antiperiodic_signs(Nt)
        # the chemical potential multiplies every time hop by e^{delta mu}
        self.fmu = math.exp(self.delta * self.mu)
        if mode == "dense-E":
            self.E = self.fmu * hopping_exponential(L, self.dk)
        elif mode == "expm":
            self.E = None
            self.Ks = (self.dk * hopping_matrix_sparse(L)).tocsc()
        else:
            raise ValueError(mode)

    # E acting on a [..., V] complex array along the last axis
    def apply_E(self, v: np.ndarray) -> np.ndarray:
        shp = v.shape
        flat = np.ascontiguousarray(v.reshape(-1, self.V))
        cols = np.concatenate([flat.real, flat.imag], axis=0).T      # V x 2m, real
        if self.mode == "dense-E":
            out = self.E @ cols
        else:
            out = self.fmu * spla.expm_multiply(self.Ks, cols)
        m = flat.shape[0]
        res = (out[:, :m] + 1j * out[:, m:]).T
        return res.reshape(shp)

    def _shape(self, v):
        v = np.asarray(v, dtype=np.complex128)
        return v.reshape(-1, self.Nt, self.V), v.shape

    def apply_M(self, phi: np.ndarray, v: np.ndarray) -> np.ndarray:
        """(M v)_t = v_t - B_t E (e^{i phi_{t-1}} * v_{t-1})."""
        vv, shp = self._shape(v)
        src = np.roll(np.exp(1j * phi)[None] * vv, 1, axis=1)      # slot t holds slice t-1
        hop = self.apply_E(src)
        out = vv - self.B[None, :, None] * hop
        return out.reshape(shp)

    def apply_Mdag(self, phi: np.ndarray, v: np.ndarray) -> np.ndarray:
        """(M^dag v)_t = v_t - B_{t+1} e^{-i phi_t} * (E v_{t+1})."""
        vv, shp = self._shape(v)
        hop = np.roll(self.apply_E(vv), -1, axis=1)                 # slot t holds E v_{t+1}
        Bn = np.roll(self.B, -1)                                   # B_{t+1}
        out = vv - Bn[None, :, None] * np.exp(-1j * phi)[None] * hop
        return out.reshape(shp)

    def apply_A(self, phi, v):
        """A v = M M^dag v."""
        return self.apply_M(phi, self.apply_Mdag(phi, v))

    def dense_M(self, phi: np.ndarray) -> np.ndarray:
        """Dense N x N matrix of M (row/col index t*V + x).  Tiny lattices only."""
        if self.E is None:
            raise ValueError("dense_M needs mode dense-E")
        V, Nt = self.V, self.Nt
        M = np.eye(self.N, dtype=np.complex128)
        for t in range(Nt):
            tp = (t - 1) % Nt
            blk = -self.B[t] * self.E * np.exp(1j * phi[tp])[None, :]
            M[t * V:(t + 1) * V, tp * V:(tp + 1) * V] += blk
        return M


# --------------------------------------------------------------------------- solver
def cg_solve(op: HubbardOperator, phi: np.ndarray, chi: np.ndarray, tol: float = 1e-12,
             max_iter: int = 100000, x0: np.ndarray | None = None):
    """Textbook (Hestenes-Stiefel) conjugate gradients on A = M M^dag, x0 = 0.

    The paper names no solver; CG is the standard method for the Hermitian
    positive definite system (M M^dag) x = chi in the effective Hamiltonian
    (Sec. 2, eq. "hamiltonian").  Each right-hand side (leading axis) is solved
    independently.  Returns x, iteration counts and true relative residuals
    ||chi - A x|| / ||chi||.
    """
    chi = np.asarray(chi, dtype=np.complex128).reshape(-1, op.Nt, op.V)
    xs, its, res = [], [], []
    for c in chi:
        x = np.zeros_like(c) if x0 is None else np.array(x0, dtype=np.complex128).reshape(c.shape)
        r = c - op.apply_A(phi, x) if x0 is not None else c.copy()
        p = r.copy()
        rr = np.vdot(r, r).real
        cc = np.vdot(c, c).real
        it = 0
        while rr > tol * tol * cc and it < max_iter:
            q = op.apply_A(phi, p)
            alpha = rr / np.vdot(p, q).real
            x = x + alpha * p
            r = r - alpha * q
            rr_new = np.vdot(r, r).real
            p = r + (rr_new / rr) * p
            rr = rr_new
            it += 1
        true = np.linalg.norm(c - op.apply_A(phi, x)) / math.sqrt(cc)
        xs.append(x)
        its.append(it)
        res.append(true)
    return np.stack(xs), np.array(its), np.array(res)


def dense_solve(op: HubbardOperator, phi: np.ndarray, chi: np.ndarray) -> np.ndarray:
    """x = (M M^dag)^{-1} chi by a dense LU solve (tiny lattices)."""
    M = op.dense_M(phi)
    A = M @ M.conj().T
    chi = np.asarray(chi, dtype=np.complex128).reshape(-1, op.N)
    x = np.linalg.solve(A, chi.T).T
    return x.reshape(-1, op.Nt, op.V)


# --------------------------------------------------------------------------- action & force
def action(chi: np.ndarray, x: np.ndarray) -> float:
    """Pseudofermion action S = Re chi^dag x with x = (M M^dag)^{-1} chi (eq. "hamiltonian"),
    summed over right-hand sides."""
    return float(np.vdot(np.asarray(chi).ravel(), np.asarray(x).ravel()).real)


def force(op: HubbardOperator, phi: np.ndarray, x: np.ndarray) -> np.ndarray:
    """dS/dphi of S = chi^dag (M M^dag)^{-1} chi, matrix-free, summed over right-hand sides.

    With A = M M^dag and x = A^{-1} chi, dS = -x^dag (dM M^dag + M dM^dag) x
    = -2 Re(x^dag dM y), y = M^dag x.  phi_{t,z} enters only block (t+1, t) of M,
    column z: dM/dphi_{t,z} e_{(t,z)} = -B_{t+1} * i e^{i phi_{t,z}} E[:, z] placed in
    slice t+1.  Hence x^dag dM y = -B_{t+1} i e^{i phi_{t,z}} y_{t,z} conj((E x_{t+1})_z).
    Returns float64 [Nt, V].
    """
    xx = np.asarray(x, dtype=np.complex128).reshape(-1, op.Nt, op.V)
    g = np.zeros((op.Nt, op.V))
    Bn = np.roll(op.B, -1)[:, None]                      # B_{t+1}
    for xr in xx:
        y = op.apply_Mdag(phi, xr)
        w_next = np.roll(op.apply_E(xr), -1, axis=0)     # slot t holds E x_{t+1}
        xdMy = -Bn * 1j * np.exp(1j * phi) * y * np.conj(w_next)
        g += -2.0 * xdMy.real
    return g


def force_dense(op: HubbardOperator, phi: np.ndarray, x: np.ndarray) -> np.ndarray:
    """dS/dphi from explicitly assembled dM matrices: g = -x^dag (dM M^dag + M dM^dag) x.

    Tiny lattices only (one dense N x N derivative matrix per field entry).
    """
    M = op.dense_M(phi)
    V, Nt = op.V, op.Nt
    xx = np.asarray(x, dtype=np.complex128).reshape(-1, op.N)
    Mh_x = [M.conj().T @ xr for xr in xx]          # M^dag x
    xh_M = [xr.conj() @ M for xr in xx]            # x^dag M
    g = np.zeros(op.N)
    dM = np.zeros((op.N, op.N), dtype=np.complex128)
    for t in range(Nt):
        tn = (t + 1) % Nt
        Bn = op.B[tn]
        for z in range(V):
            c = t * V + z
            dM[tn * V:(tn + 1) * V, c] = -Bn * 1j * np.exp(1j * phi[t, z]) * op.E[:, z]
            tot = 0.0
            for xr, a, b in zip(xx, Mh_x, xh_M):
                # x^dag dM (M^dag x) + (x^dag M) dM^dag x
                tot += (xr.conj() @ (dM @ a) + b @ (dM.conj().T @ xr)).real
            g[c] = -tot
            dM[tn * V:(tn + 1) * V, c] = 0.0
    return g.reshape(Nt, V)


# --------------------------------------------------------------------------- linear form
class LinearHubbardOperator:
    """The fermion matrix exactly as printed in eq. "ferm_op" (Sec. 2), linear in delta*kappa:

        M^AA_{(x,t)(y,t')} = delta_xy (delta_{t+1,t'} - delta_{tt'} e^{i phi_{x,t}})
        M^BB_{(x,t)(y,t')} = delta_xy (delta_{tt'} - delta_{t-1,t'} e^{-i phi_{x,t}})
        M^AB = M^BA      = -delta kappa delta_<x,y> delta_{tt'}

    with phi = delta * the paper's field (so e^{i delta phi_paper} = e^{i phi}) and
    antiperiodic time: a hop across the wrap carries -1 (B_t below).
    """

    def __init__(self, L: int, Nt: int, beta: float, kappa: float = 1.0):
        self.L, self.Nt, self.beta, self.kappa = L, Nt, float(beta), float(kappa)
        self.V = 2 * L * L
        self.N = self.V * Nt
        self.delta = self.beta / Nt
        self.dk = self.delta * self.kappa
        self.nA = L * L
        self.B = antiperiodic_signs(Nt)
        self.K = hopping_matrix_sparse(L).tocsr()

    def _shape(self, v):
        v = np.asarray(v, dtype=np.complex128)
        return v.reshape(-1, self.Nt, self.V), v.shape

    def _hop(self, vv):
        flat = vv.reshape(-1, self.V)
        return (self.K @ flat.T).T.reshape(vv.shape)

    def apply_M(self, phi, v):
        vv, shp = self._shape(v)
        A, Bs = slice(0, self.nA), slice(self.nA, self.V)
        Bn = np.roll(self.B, -1)[None, :, None]                     # B_{t+1}
        nxt = Bn * np.roll(vv, -1, axis=1)                          # v_{t+1} across the wrap
        prv = self.B[None, :, None] * np.roll(vv, 1, axis=1)       # v_{t-1} across the wrap
        out = np.empty_like(vv)
        out[..., A] = nxt[..., A] - np.exp(1j * phi[:, A])[None] * vv[..., A]
        out[..., Bs] = vv[..., Bs] - np.exp(-1j * phi[:, Bs])[None] * prv[..., Bs]
        out -= self.dk * self._hop(vv)
        return out.reshape(shp)

    def apply_Mdag(self, phi, v):
        vv, shp = self._shape(v)
        A, Bs = slice(0, self.nA), slice(self.nA, self.V)
        Bn = np.roll(self.B, -1)[None, :, None]
        prv = self.B[None, :, None] * np.roll(vv, 1, axis=1)       # B_t v_{t-1}
        nxt = Bn * np.roll(vv, -1, axis=1)                          # B_{t+1} v_{t+1}
        ph_next = np.roll(phi, -1, axis=0)                          # phi_{t+1}
        out = np.empty_like(vv)
        out[..., A] = prv[..., A] - np.exp(-1j * phi[:, A])[None] * vv[..., A]
        out[..., Bs] = vv[..., Bs] - np.exp(1j * ph_next[:, Bs])[None] * nxt[..., Bs]
        out -= self.dk * self._hop(vv)
        return out.reshape(shp)

    def apply_A(self, phi, v):
        return self.apply_M(phi, self.apply_Mdag(phi, v))

    def dense_M(self, phi):
        """Entry by entry from eq. "ferm_op" (tiny lattices)."""
        V, Nt, nA = self.V, self.Nt, self.nA
        M = np.zeros((self.N, self.N), dtype=np.complex128)
        K = self.K.toarray()
        for t in range(Nt):
            for x in range(V):
                r = t * V + x
                if x < nA:
                    tn = (t + 1) % Nt
                    M[r, tn * V + x] += self.B[tn]
                    M[r, r] -= np.exp(1j * phi[t, x])
                else:
                    tp = (t - 1) % Nt
                    M[r, r] += 1.0
                    M[r, tp * V + x] -= self.B[t] * np.exp(-1j * phi[t, x])
            M[t * V:(t + 1) * V, t * V:(t + 1) * V] -= self.dk * K
        return M

    def dense_dM(self, phi, t, x):
        """d M / d phi_{t,x} as a dense matrix (one nonzero entry)."""
        dM = np.zeros((self.N, self.N), dtype=np.complex128)
        V = self.V
        if x < self.nA:
            dM[t * V + x, t * V + x] = -1j * np.exp(1j * phi[t, x])
        else:
            tp = (t - 1) % self.Nt
            dM[t * V + x, tp * V + x] = 1j * self.B[t] * np.exp(-1j * phi[t, x])
        return dM


def force_linear(op: LinearHubbardOperator, phi, x) -> np.ndarray:
    """dS/dphi for the linear form, -2 Re(x^dag dM y) with y = M^dag x, summed over rhs.

    phi_{t,z} enters one entry of M: the diagonal -e^{i phi} on A sites, the entry
    -B_t e^{-i phi} coupling slice t-1 on B sites.
    """
    xx = np.asarray(x, dtype=np.complex128).reshape(-1, op.Nt, op.V)
    g = np.zeros((op.Nt, op.V))
    A, Bs = slice(0, op.nA), slice(op.nA, op.V)
    for xr in xx:
        y = op.apply_Mdag(phi, xr)
        yprev = np.roll(y, 1, axis=0)                               # y_{t-1} (unsigned)
        gA = -2.0 * (np.exp(1j * phi[:, A]) * np.conj(xr[:, A]) * y[:, A]).imag
        gB = 2.0 * op.B[:, None] * (np.exp(-1j * phi[:, Bs]) * np.conj(xr[:, Bs]) * yprev[:, Bs]).imag
        g[:, A] += gA
        g[:, Bs] += gB
    return g


def force_dense_linear(op: LinearHubbardOperator, phi, x) -> np.ndarray:
    """-x^dag (dM M^dag + M dM^dag) x from dense derivatives (tiny lattices)."""
    M = op.dense_M(phi)
    xx = np.asarray(x, dtype=np.complex128).reshape(-1, op.N)
    g = np.zeros(op.N)
    for t in range(op.Nt):
        for z in range(op.V):
            dM = op.dense_dM(phi, t, z)
            dA = dM @ M.conj().T + M @ dM.conj().T
            g[t * op.V + z] = -sum(np.vdot(xr, dA @ xr).real for xr in xx)
    return g.reshape(op.Nt, op.V)


def dense_solve_op(op, phi, chi):
    """x = (M M^dag)^{-1} chi by a dense solve, for any operator with dense_M."""
    M = op.dense_M(phi)
    A = M @ M.conj().T
    chi = np.asarray(chi, dtype=np.complex128).reshape(-1, op.N)
    return np.linalg.solve(A, chi.T).T.reshape(-1, op.Nt, op.V)


# --------------------------------------------------------------------------- Sec. 3 weight
def log_det(op: HubbardOperator, phi: np.ndarray) -> tuple[float, float]:
    """(log|det M[phi]|, arg det M[phi]) of the exponential form, from the block-cyclic identity
    det M = det(1 + E D_{Nt-1} ... E D_0) (antiperiodic wrap): the product is built slice by
    slice with the dense E and its determinant taken by LU (numpy's slogdet).  Tiny and small
    lattices (dense V x V); the product is not stabilised, so beta (3|kappa| + |mu|) must stay
    moderate.  The argument is reduced to (-pi, pi]."""
    if op.E is None:
        raise ValueError("log_det needs mode dense-E")
    P = np.eye(op.V, dtype=complex)
    for t in range(op.Nt):
        P = op.E @ (np.exp(1j * phi[t])[:, None] * P)
    s, ld = np.linalg.slogdet(np.eye(op.V) + P)
    return float(ld), float(np.angle(s))


def sign_phase(op_plus: HubbardOperator, op_minus: HubbardOperator, phi: np.ndarray) -> float:
    """theta of Sec. 3: the weight det(M[phi, mu] M[phi, -mu]^dag) = |p| e^{i theta}, so
    theta = arg det M[phi, mu] - arg det M[phi, -mu], reduced to (-pi, pi]."""
    a = log_det(op_plus, phi)[1] - log_det(op_minus, phi)[1]
    return float(np.angle(np.exp(1j * a)))


def reweight(obs: np.ndarray, theta: np.ndarray) -> complex:
    """Sec. 3 reweighting: <O>_p = <O e^{i theta}>_|p| / <e^{i theta}>_|p| over samples drawn
    with the weight |p|."""
    z = np.exp(1j * np.asarray(theta, dtype=float))
    return complex(np.mean(np.asarray(obs) * z) / np.mean(z))
