// Internal declarations shared by the host ABI, the tables and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

#include "hub.h"
#include "hub_tables.hpp"

namespace hub {

constexpr int kNumCounters = 8;    // last-block counters, one per kernel role

// Per-right-hand-side CG scalars kept on the device (all FP64).
struct CgScalars {
    double rr;        // ||r||^2 of the iterated residual
    double alpha;
    double beta;
    double tt;        // ||M^dag p||^2
    double chichi;    // ||chi||^2
    double true_rr;   // ||chi - A x_hi||^2 at the last reliable update
    double tol2;      // tol^2 * ||chi||^2
    double rec_rr;    // iterated ||r||^2 just before the last reliable update
    double rr_last;   // ||r_i||^2 that the last iteration which did work started from
    int32_t active;   // unused (kept for layout)
    int32_t done;     // 1 once the true residual met tol
    int32_t iters;
    int32_t reliable;
    int32_t nonfinite;
    int32_t x_pending;   // paired x updates: the last iteration left alpha_prev * p for x
    double alpha_prev;   // that iteration's alpha
};

}  // namespace hub

struct hub_ctx {
    int device = 0;
    int L = 0, Nt = 0, V = 0, nrhs_max = 0;
    long long N = 0;                 // V * Nt
    double beta = 0, kappa = 0, delta = 0, mu = 0;
    int path = HUB_PATH_FUSED;
    int form = HUB_FORM_EXP;
    bool specialized = true;         // use a compile-time-L kernel when one exists
    bool split_forced = false;       // HUB_PATH_SPLIT requested: no fused kernel of any kind
    bool poly = false;               // FP32 operators by the polynomial stencil (HUB_PATH_AUTO, L = 51, 102)
    double poly_a0 = 1.0;            // its polynomial (exp_poly_ratios): a_0, a_k / a_{k-1}, error bound
    double poly_ratio[11] = {};
    double poly_err = -1.0;
    bool poly64 = false;             // FP64 operators by the polynomial stencil (HUB_PATH_AUTO, L = 102)
    double poly64_a0 = 1.0;          // and its polynomial
    double poly64_ratio[11] = {};
    double poly64_err = -1.0;
    int lds_fused64 = 0, lds_fused32 = 0;
    int max_lds = 0;
    hub::FftPlan plan{};

    // tables
    double* roots64 = nullptr;   // [L][2]
    float* roots32 = nullptr;
    double* etab64 = nullptr;    // [L*L][4]
    float* etab32 = nullptr;

    // reductions
    double* partials = nullptr;          // [nrhs_max * max_blocks_per_rhs]
    int max_partials = 0;
    unsigned int* counters = nullptr;    // [kNumCounters]
    double* red_out = nullptr;           // scratch scalar outputs

    // split-path workspace: one complex vector per right-hand side
    void* split_w = nullptr;             // complex128 [nrhs_max][N] (reused as complex64)

    // CG workspace (allocated on first solve)
    bool cg_ready = false;
    void* cg_rhi = nullptr;      // complex128
    void* cg_tmp = nullptr;      // complex128 (M^dag x_hi)
    void* cg_x = nullptr;        // complex128 (FP64 mode) or complex64 (mixed)
    void* cg_r = nullptr;
    void* cg_p = nullptr;
    void* cg_t = nullptr;
    void* ph64 = nullptr;        // e^{i phi} complex128 [Nt][V] for the solve in progress
    void* ph32 = nullptr;        // e^{i phi} complex64 [Nt][V]
    hub::CgScalars* scal = nullptr;      // device [nrhs_max]
    double* cg_pr = nullptr;             // ||r||^2 partials, [3][nrhs_max][max_partials]
    double* cg_pt = nullptr;             // ||M^dag p||^2 partials, [nrhs_max][max_partials]
    hub::CgScalars* scal_host = nullptr; // pinned host mirror
    hipEvent_t cg_event = nullptr;       // marks the copy of the scalars into scal_host
    // persistent CG launches (FP32 iterations of the L = 102 sublattice kernel)
    unsigned* persist_bar = nullptr;     // device [4]: arrivals, generation, abort flag
    unsigned* persist_flag_host = nullptr;   // pinned mirror of the abort flag
    int persist_mode = 0;                // 1: use when co-resident, 0: never (the default)
    bool persist_ok = true;              // false once a cooperative launch was refused
    long long persist_spin = 1LL << 24;  // polls before a barrier wait gives up
    int persist_grid = -1;               // co-resident workgroups (-1: not yet known)
    long long persist_launches = 0;      // during the current solve
    // HMC trajectory workspace (allocated on the first trajectory)
    void* tr_chi = nullptr;              // complex128 [nrhs_max][N]: the pseudofermions
    void* tr_x = nullptr;                // complex128 [nrhs_max][N]: the solutions
    double* tr_pi = nullptr;             // [N] momenta
    double* tr_phi0 = nullptr;           // [N] the field at the start
    double* tr_g = nullptr;              // [N] dS_f/dphi
    double* tr_E = nullptr;              // [2] device: boson energy, action
    double* tr_E_host = nullptr;         // [2] pinned mirror
    double* force_tmp = nullptr;         // [nrhs_max][N] doubles, per-rhs force before summation (hub_create)
    // log det workspace (allocated on the first hub_log_det): two V x V complex128 matrices
    void* ld_x = nullptr;
    void* ld_y = nullptr;
};
