/*
 * hub.h - C ABI of the MI355X (gfx950) honeycomb Hubbard-model HMC hot path.
 *
 * The library applies the fermion matrix M[phi] of the Hubbard-Stratonovich
 * transformed Hubbard model on the honeycomb lattice (paper Sec. 2, eq. "ferm_op"
 * in its exponential transfer-matrix form), solves (M M^dag) x = chi with
 * conjugate gradients, and computes the pseudofermion force dS/dphi of
 * S = chi^dag (M M^dag)^{-1} chi (Sec. 2, eq. "hamiltonian").
 *
 * Two forms of the operator are available (hub_params.form).  HUB_FORM_EXP, the default:
 * the exponential transfer-matrix form.  Operator (all indices mod Nt,
 * E = e^{delta mu} exp(delta*kappa*K), delta = beta/Nt; the
 * chemical potential mu is 0 at half filling, and the weight of Sec. 3 away from it is
 * det(M[phi,mu] M[phi,-mu]^dag)):
 *     (M v)_t     = v_t - B_t     E (e^{i phi_{t-1}} * v_{t-1})
 *     (M^dag v)_t = v_t - B_{t+1} e^{-i phi_t} * (E v_{t+1})
 * with B_0 = -1 (antiperiodic wrap) and B_t = +1 otherwise.  K is the
 * nearest-neighbour hopping matrix of the L x L honeycomb torus (Sec. 1,
 * fig. "honeycomb_lattice"): A(n) is bonded to B(n), B(n-e1), B(n-e2).
 *
 * HUB_FORM_LINEAR: eq. "ferm_op" exactly as printed, linear in delta*kappa (mu must be 0):
 *     A sites: (M v)_{t,x} = B_{t+1} v_{t+1,x} - e^{i phi_{t,x}} v_{t,x}   - dk (K v_t)_x
 *     B sites: (M v)_{t,x} = v_{t,x} - B_t e^{-i phi_{t,x}} v_{t-1,x}       - dk (K v_t)_x
 * with dk = delta*kappa; M^dag is its conjugate transpose.  Every entry point below
 * works for both forms; the solver, the action and the HMC updates are form-independent.
 *
 * Layouts (C-contiguous, fastest index last):
 *     site x = s*L*L + n1*L + n2      (s = 0 for sublattice A, 1 for B)
 *     V = 2*L*L sites per slice, N = V*Nt entries per vector
 *     phi    : double [Nt][V]                     (float for the *_c64 calls)
 *     vectors: complex128 [nrhs][Nt][V], interleaved (re, im) doubles
 *              (complex64 [nrhs][Nt][V] for the *_c64 calls)
 *     force  : double [Nt][V]
 *
 * Ownership: every array argument is a DEVICE pointer on the context's device,
 * owned by the caller; the library keeps no pointer after a call returns.  The
 * context owns its tables and workspace: hub_create allocates the tables, the
 * reduction partials and the operator scratch, the first hub_cg_solve the solver
 * vectors, the first hub_trajectory its own vectors, the first hub_log_det its two
 * matrices; nothing else allocates;
 * hub_destroy frees all of it.
 *
 * Streams: every call enqueues its work on `stream` (a hipStream_t; NULL means
 * the default stream) and returns without synchronising, except hub_cg_solve,
 * which synchronises on `stream` to read its convergence status.
 *
 * Errors: calls return a hub_status and never abort.  Arguments are validated
 * before anything is launched; hub_last_error() returns a thread-local message
 * describing the last non-OK status of the calling thread.
 *
 * Threads: a context may be used from one host thread at a time.  Calls on one
 * context that overlap in time (on different streams) share its workspace and race.
 *
 * Devices: a context belongs to the device that was current at hub_create; every
 * later call must be made with that device current (HUB_ERR_ARG otherwise), except
 * hub_destroy, which switches to it by itself.
 */
#ifndef HUB_H
#define HUB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hub_ctx hub_ctx;

typedef enum {
    HUB_OK = 0,
    HUB_ERR_ARG = 1,        /* invalid argument (null pointer, size, aliasing, option) */
    HUB_ERR_DEVICE = 2,     /* a HIP runtime call failed                               */
    HUB_ERR_NOMEM = 3,      /* device allocation failed                                */
    HUB_ERR_NOCONV = 4,     /* CG stopped (max_iter, stagnation) before meeting tol     */
    HUB_ERR_NONFINITE = 5   /* NaN or Inf appeared in a CG scalar                      */
} hub_status;

typedef enum { HUB_PREC_FP64 = 0, HUB_PREC_MIXED = 1 } hub_prec;

/* Which kernel layout applies E: AUTO picks the fused one-slice-per-workgroup
 * kernel when a slice fits in LDS, else the three-kernel split path, and at L = 51 or 102 with
 * 3 |delta kappa| <= 0.25 the polynomial stencil for the FP32 operators (see hub_apply_M_c64),
 * at L = 102 for the FP64 ones too where its bound allows (see hub_apply_M).  FUSED and SPLIT
 * force one (FUSED fails with HUB_ERR_ARG when the slice does not fit); both apply E through
 * the transforms in both precisions. */
typedef enum { HUB_PATH_AUTO = 0, HUB_PATH_FUSED = 1, HUB_PATH_SPLIT = 2 } hub_path;

/* Which fermion matrix the context applies (see the top of this file). */
typedef enum { HUB_FORM_EXP = 0, HUB_FORM_LINEAR = 1 } hub_form;

typedef struct {
    int32_t L;          /* torus extent, 1 <= L <= 1024; HUB_FORM_EXP: every prime factor <= 17   */
    int32_t Nt;         /* time slices, Nt >= 1                                                 */
    double beta;        /* inverse temperature, delta = beta/Nt; any finite value              */
    double kappa;       /* hopping amplitude; any finite value, either sign (with -kappa and
                           -phi the context applies the hole operator M[-phi, -kappa], Sec. 2)  */
    int32_t nrhs_max;   /* largest nrhs any call on this context will pass, >= 1; nrhs_max * N
                           < 2^40 and each launch grid (about 2 * nrhs_max * Nt blocks) within
                           2^31 - 1, else HUB_ERR_ARG                                            */
    int32_t path;       /* hub_path                                                              */
    double mu;          /* chemical potential: every time hop carries e^{delta mu} (0 = half filling) */
    int32_t form;       /* hub_form; HUB_FORM_LINEAR ignores `path` and requires mu == 0       */
} hub_params;

typedef struct {
    double tol;             /* stop when ||chi - M M^dag x|| <= tol ||chi|| (true FP64 residual) */
    int32_t max_iter;       /* iteration cap per right-hand side, >= 1                          */
    int32_t reliable_every; /* FP64 residual recomputation every this many iterations, >= 1     */
    int32_t prec;           /* hub_prec: FP64 throughout, or FP32 inner iterations               */
    int32_t use_x0;         /* 1: x holds the initial guess on entry; 0: start from x = 0       */
    int32_t stall_updates;  /* > 0: stop with HUB_ERR_NOCONV once, for every unfinished
                               right-hand side, this many consecutive reliable updates found the
                               iterated residual below tol but no 1 % gain on the best true
                               residual (the attainable-accuracy floor); 0: off               */
    double* history_host;   /* optional (NULL: off), HOST memory [nrhs][history_len]: the true
                               relative residual ||chi - A x|| / ||chi|| after each reliable update
                               of right-hand side r at history_host[r * history_len + j], j = 0, 1, ..;
                               entries past hub_cg_info.reliable_updates (or history_len) untouched */
    int32_t history_len;    /* entries per right-hand side in history_host, >= 0                    */
} hub_cg_opts;

typedef struct {
    int32_t iters;              /* CG iterations performed for this right-hand side           */
    int32_t reliable_updates;   /* FP64 residual recomputations                               */
    double true_rel_res;        /* ||chi - A x|| / ||chi|| in FP64 at exit                    */
    double recursive_rel_res;   /* the iterated residual's ||r|| / ||chi|| at exit            */
    int32_t persistent_launches;/* persistent launches of the solve (hub_set_cg_launch), the same
                                   in every entry; 0: two launches per iteration                 */
} hub_cg_info;

/* Create a context on the current HIP device: for HUB_FORM_EXP builds the momentum-space
 * hopping table E(k) (Sec. 1: bands +-kappa|f(k)|) and the DFT roots of unity in FP64.
 * `stream` is used for the table uploads.  *out is set to NULL on failure. */
hub_status hub_create(const hub_params* params, void* stream, hub_ctx** out);

/* Release every device allocation of the context (synchronises the device).  NULL is a no-op. */
void hub_destroy(hub_ctx* ctx);

/* out = M[phi] in  (Sec. 2, eq. "ferm_op", in the context's form), FP64.
 * in and out: complex128 [nrhs][Nt][V]; out may overlap neither in nor phi (HUB_ERR_ARG).
 * 1 <= nrhs <= nrhs_max.  With HUB_PATH_AUTO at L = 102 E is applied as e^{delta mu}
 * p(delta kappa K), p the degree-9 truncated Chebyshev series of e^z on [-3|delta kappa|,
 * 3|delta kappa|], when its error bound is at most 4e-17 (2.9e-17 at 3|delta kappa| = 0.1875,
 * below FP64 rounding); otherwise, and at every other L, through the per-slice transforms.
 * The same holds for every FP64 operator of the context (hub_apply_Mdag, the FP64 steps of
 * hub_cg_solve, hub_force and the slab variants). */
hub_status hub_apply_M(hub_ctx* ctx, const double* phi, const void* in, void* out,
                       int32_t nrhs, void* stream);

/* out = M[phi]^dag in, FP64.  Same layout and rules as hub_apply_M. */
hub_status hub_apply_Mdag(hub_ctx* ctx, const double* phi, const void* in, void* out,
                          int32_t nrhs, void* stream);

/* FP32 variants of the two operators (complex64 vectors, float phi): the kernels
 * that the mixed-precision CG iterates with.  With HUB_PATH_AUTO at L = 51 or 102 and
 * 3 |delta kappa| <= 0.25 they apply E = e^{delta mu} exp(delta kappa K) (Sec. 2, eq.
 * "ferm_op") as e^{delta mu} p(delta kappa K), p the degree-5 truncated Chebyshev series of e^z on
 * [-3|delta kappa|, 3|delta kappa|] (K's spectrum lies in [-3, 3]), an error of at most 1.1e-8
 * relative, below FP32 rounding; otherwise through the per-slice transforms (for the FP64
 * entry points see hub_apply_M). */
hub_status hub_apply_M_c64(hub_ctx* ctx, const float* phi, const void* in, void* out,
                           int32_t nrhs, void* stream);
hub_status hub_apply_Mdag_c64(hub_ctx* ctx, const float* phi, const void* in, void* out,
                              int32_t nrhs, void* stream);

/* Time slabs: the operators and the force on one shard of a time-sharded vector (the layout a
 * run that splits the Nt slices over several GPUs gives each of them; Sec. 2 operator,
 * HUB_FORM_EXP only, else HUB_ERR_ARG).  The slab is the nt consecutive slices t0 .. t0+nt-1 of
 * the context's Nt (0 <= t0, nt >= 1, t0 + nt <= Nt); its arrays hold those slices only:
 *     phi: double [nt][V] (float for _c64),  in, out, x: complex [nrhs][nt][V],  dSdphi: double [nt][V].
 * The one slice each needs from beyond the slab is passed as a halo (what a neighbouring shard
 * would send), one slice per right-hand side, complex [nrhs][V]:
 *     hub_apply_M_slab:    in_halo = v at slice (t0 - 1) mod Nt, phi_halo (double [V]) = phi there;
 *     hub_apply_Mdag_slab: in_halo = v at slice (t0 + nt) mod Nt;
 *     hub_force_slab:      x_halo  = x at slice (t0 + nt) mod Nt.
 * Row t of the output is row t0 + t of the full operator (or force); with t0 = 0, nt = Nt and the
 * halo taken from the vector itself the calls reproduce hub_apply_M, hub_apply_Mdag and hub_force.
 * The antiperiodic sign follows the global slice index.  out may overlap no input or halo. */
hub_status hub_apply_M_slab(hub_ctx* ctx, int32_t t0, int32_t nt, const double* phi, const void* in,
                            const double* phi_halo, const void* in_halo, void* out, int32_t nrhs, void* stream);
hub_status hub_apply_Mdag_slab(hub_ctx* ctx, int32_t t0, int32_t nt, const double* phi, const void* in,
                               const void* in_halo, void* out, int32_t nrhs, void* stream);
hub_status hub_apply_M_slab_c64(hub_ctx* ctx, int32_t t0, int32_t nt, const float* phi, const void* in,
                                const float* phi_halo, const void* in_halo, void* out, int32_t nrhs, void* stream);
hub_status hub_apply_Mdag_slab_c64(hub_ctx* ctx, int32_t t0, int32_t nt, const float* phi, const void* in,
                                   const void* in_halo, void* out, int32_t nrhs, void* stream);
hub_status hub_force_slab(hub_ctx* ctx, int32_t t0, int32_t nt, const double* phi, const void* x,
                          const void* x_halo, double* dSdphi, int32_t nrhs, void* stream);

/* Solve (M M^dag) x = chi for nrhs independent right-hand sides (Sec. 2, eq.
 * "hamiltonian": the pseudofermion term needs (M M^dag)^{-1} chi).  Conjugate
 * gradients from x0 = 0 (or x on entry when opts->use_x0), all reductions in FP64.
 * With opts->prec == HUB_PREC_MIXED the iterations run in FP32 and every
 * reliable_every iterations the FP64 solution is updated and the FP64 residual
 * recomputed (in both precisions; a right-hand side whose iterated residual meets tol
 * earlier idles until then).  Convergence is always judged on the true FP64 residual.
 * Every reduction has a fixed order, so repeating a call gives bitwise the same x and info.
 * Each right-hand side has its own scalars and schedule; solved in a batch it gives bitwise the
 * result of solving it alone whenever both launches use the same kernel variant (at L = 51 the
 * variant changes where nrhs * Nt crosses 256 slices).
 * chi, x: complex128 [nrhs][Nt][V]; x may overlap neither chi nor phi.  info_host: nrhs entries
 * in HOST memory (may be NULL).  Returns HUB_ERR_NOCONV (x = last FP64 iterate,
 * info filled) at max_iter or on stagnation (opts->stall_updates), or
 * HUB_ERR_NONFINITE when the iteration breaks down. */
hub_status hub_cg_solve(hub_ctx* ctx, const double* phi, const void* chi, void* x, int32_t nrhs,
                        const hub_cg_opts* opts, hub_cg_info* info_host, void* stream);

/* dS/dphi of the pseudofermion action S = sum_r chi_r^dag x_r, x_r = (M M^dag)^{-1} chi_r,
 * from the solutions x (complex128 [nrhs][Nt][V]).  HUB_FORM_EXP:
 *     dSdphi[t][z] = sum_r -2 B_{t+1} Im( e^{i phi_{t,z}} x_{r,t,z} conj((E x_{r,t+1})_z) ).
 * HUB_FORM_LINEAR, with y_r = M^dag x_r:
 *     A sites: dSdphi[t][z] = sum_r -2 Im( e^{i phi_{t,z}} conj(x_{r,t,z}) y_{r,t,z} )
 *     B sites: dSdphi[t][z] = sum_r 2 B_t Im( e^{-i phi_{t,z}} conj(x_{r,t,z}) y_{r,t-1,z} ).
 * dSdphi (double [Nt][V]) is overwritten and may overlap neither x nor phi.  The Gaussian
 * term phi/(delta U) is the caller's. */
hub_status hub_force(hub_ctx* ctx, const double* phi, const void* x, double* dSdphi,
                     int32_t nrhs, void* stream);

/* hub_force for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same kernels and the same result
 * as hub_force, bit for bit, but the per-right-hand-side forces are summed through the
 * library's static device scratch instead of the context's buffer.  Calls no allocating
 * routine.  The scratch holds at most 2^23 doubles (64 MiB): nrhs * N above that returns
 * HUB_ERR_ARG (one right-hand side, or HUB_FORM_LINEAR, uses no scratch and has no limit).
 * Every call on one GPU shares that GPU's scratch: calls that overlap in time on one GPU
 * (from any context, stream or thread) race.  Each call writes every scratch entry it reads;
 * nothing needs clearing. */
hub_status hub_force_noalloc(hub_ctx* ctx, const double* phi, const void* x, double* dSdphi,
                             int32_t nrhs, void* stream);

/* S_dev[0] = sum_r Re(chi_r^dag x_r) in FP64 (the pseudofermion action of eq.
 * "hamiltonian" when x solves M M^dag x = chi).  S_dev: one double on the device. */
hub_status hub_action(hub_ctx* ctx, const void* chi, const void* x, int32_t nrhs,
                      double* S_dev, void* stream);

/* One molecular-dynamics update of an HMC trajectory (Sec. 2: phi evolves with the
 * momentum pi under H = pi^2/2 + phi^2/(2 delta U) + S_f[phi]).  With the total force
 * F = phi/(delta U) + dSdphi (dSdphi from hub_force):  pi -= eps_pi * F,  then
 * phi += eps_phi * pi.  phi, pi, dSdphi: double [Nt][V] on the device, not overlapping;
 * phi and pi are updated in place.  A leapfrog step is (eps/2, eps), (eps, eps), ...,
 * (eps/2, 0).  U > 0. */
hub_status hub_md_update(hub_ctx* ctx, double* phi, double* pi, const double* dSdphi, double U,
                         double eps_pi, double eps_phi, void* stream);

/* out_dev[0] = sum pi^2/2 + sum phi^2/(2 delta U) in FP64: the bosonic part of the HMC
 * Hamiltonian of eq. "hamiltonian" (its fermionic part is hub_action).  One double on the device. */
hub_status hub_boson_energy(hub_ctx* ctx, const double* phi, const double* pi, double U, double* out_dev,
                            void* stream);

/* Molecular-dynamics integrators of hub_trajectory. */
typedef enum { HUB_MD_LEAPFROG = 0, HUB_MD_OMELYAN = 1 } hub_integrator;

typedef struct {
    double U;               /* on-site coupling of the Gaussian term phi^2/(2 delta U), > 0        */
    double eps;             /* molecular-dynamics step, > 0                                         */
    int32_t n_md;           /* steps per trajectory, >= 1                                           */
    int32_t integrator;     /* hub_integrator: leapfrog (n_md + 1 forces) or the second-order
                               minimum-norm scheme of Omelyan, Mryglod and Folk (2 n_md + 1)         */
    hub_cg_opts cg;         /* every solve of the trajectory; use_x0 and the history are ignored
                               (the first solve starts from 0, the others from the previous one)   */
} hub_traj_opts;

typedef struct {
    int32_t accepted;       /* 1: phi holds the end of the trajectory; 0: phi was restored          */
    int32_t n_forces;       /* force evaluations, one per CG solve (the first also serves H0)      */
    int32_t cg_iters;       /* CG iterations over all solves, largest right-hand side count each    */
    double H0, H1, dH;      /* Hamiltonian at the start and end (FP64), dH = H1 - H0                */
} hub_traj_info;

/* One HMC trajectory (Sec. 2) on the device: heat bath chi = M[phi] rho for nrhs
 * pseudofermions, molecular dynamics of H = pi^2/2 + phi^2/(2 delta U) + sum_r chi_r^dag
 * (M M^dag)^{-1} chi_r with the adjoint force, and the Metropolis decision: accepted when
 * dH <= 0 or u < e^{-dH}.  phi (double [Nt][V]) is updated in place and restored when the
 * trajectory is rejected or a solve fails (the status of that solve is returned).  pi0
 * (double [Nt][V]) and rho (complex128 [nrhs][Nt][V]) are inputs on the device, not
 * overlapping phi; u is the uniform deviate of the decision.  The random numbers are the
 * caller's: the library draws none.  The first call allocates the trajectory's vectors in
 * the context; the call synchronises on `stream` (each solve reads its status). */
hub_status hub_trajectory(hub_ctx* ctx, double* phi, const double* pi0, const void* rho, int32_t nrhs,
                          double u, const hub_traj_opts* opts, hub_traj_info* info_host, void* stream);

/* log det M[phi] of the exponential form with the context's kappa and mu (Sec. 2; Sec. 3: the
 * weight away from half filling is det(M[phi,mu] M[phi,-mu]^dag) = det M[phi,mu] conj det
 * M[phi,-mu], so its phase theta, the reweighting factor e^{i theta}, is the difference of the
 * arguments from two contexts at +mu and -mu).  Computed as det(1 + E D_{Nt-1} ... E D_0), the
 * block-cyclic identity of the antiperiodic operator: the transfer product is applied slice by
 * slice to the V columns of the identity with the library's own E kernels, then one workgroup
 * takes an LU with partial pivoting in FP64.  out_dev (two doubles on the device): out_dev[0] =
 * log|det M| (-inf for a singular product), out_dev[1] = arg det M in (-pi, pi].  Small lattices:
 * V <= 1152 (L <= 24) and |beta| (3|kappa| + |mu|) <= 29 (the product is not stabilised), else
 * HUB_ERR_ARG; HUB_FORM_EXP only.  The first call allocates two V x V complex128 matrices in the
 * context.  Stream-ordered, no synchronisation. */
hub_status hub_log_det(hub_ctx* ctx, const double* phi, double* out_dev, void* stream);

/* CG launch policy of a context.  persistent = 1: the FP32 iterations of a mixed solve with the
 * one-sublattice-at-a-time kernel (exponential form, L = 102) run as one cooperative launch per
 * block of iterations (all right-hand sides in one launch; every workgroup loops over
 * (right-hand side, slice) items, with grid barriers between the M^dag and M phases), provided
 * the device holds the whole grid at once, else as two launches per iteration of that kernel;
 * the result is the same bit for bit.  persistent = 2: always two launches per iteration of that
 * same kernel (what the persistent launch reproduces).  With 1 or 2 every FP32 operator of an
 * L = 102 context uses the sublattice kernel.  persistent = 0 (the default): two launches per
 * iteration with the context's fastest FP32 kernels (at L = 102 and 3 |delta kappa| <= 0.25 the
 * polynomial stencil, see hub_apply_M_c64), measured faster on MI355X than both.
 * barrier_spin_limit > 0 bounds every wait at a grid barrier to that many polls (0 restores the
 * default, 2^24 polls, seconds); a wait that runs out makes every workgroup leave the launch and
 * hub_cg_solve return HUB_ERR_DEVICE with x undefined. */
hub_status hub_set_cg_launch(hub_ctx* ctx, int32_t persistent, int64_t barrier_spin_limit);

/* Report the transform layout the context uses (hub_path value, never AUTO) and the
 * LDS bytes per workgroup of its transform kernel (HUB_FORM_LINEAR: FUSED and 0, one
 * stencil kernel that uses no dynamic LDS).  Where the polynomial stencil applies E instead
 * (see hub_apply_M and hub_apply_M_c64) the layout reported is the one the other operators of
 * the context use. */
hub_status hub_query(const hub_ctx* ctx, int32_t* path, int32_t* lds_bytes);

/* Thread-local description of the last non-OK status returned on this thread. */
const char* hub_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HUB_H */
