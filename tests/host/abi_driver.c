/* A plain C client of the C ABI (include/hub.h): no Python, no torch.  Reads phi and chi
 * from a binary file, runs M chi, a mixed-precision CG solve and the force on the current
 * HIP device, and writes M chi, x and dS/dphi to a binary file.
 *
 *   abi_driver L Nt beta kappa form in.bin out.bin [U eps n_md u]
 *
 * in.bin : phi (Nt*V doubles), chi (Nt*V complex doubles, interleaved), and with the
 *          trajectory arguments the momenta pi0 (Nt*V doubles)
 * out.bin: M chi (Nt*V complex), x (Nt*V complex), dSdphi (Nt*V doubles), then the CG
 *          iteration count and true relative residual (int32, double); with the trajectory
 *          arguments also one leapfrog HMC trajectory from (phi, pi0) with heat-bath vector
 *          rho = chi, uniform deviate u and solves to 1e-12: accepted (int32), dH (double), phi after it
 *          (Nt*V doubles)
 * Exit status 0 on success, 1 on a library or runtime error (message on stderr). */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "hub.h"

#define CHECK_HIP(x)                                                        \
    do {                                                                    \
        hipError_t e_ = (x);                                                \
        if (e_ != hipSuccess) {                                             \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));        \
            return 1;                                                       \
        }                                                                   \
    } while (0)

#define CHECK_HUB(x)                                                        \
    do {                                                                    \
        hub_status s_ = (x);                                                \
        if (s_ != HUB_OK) {                                                 \
            fprintf(stderr, "%s: status %d: %s\n", #x, (int)s_, hub_last_error()); \
            return 1;                                                       \
        }                                                                   \
    } while (0)

int main(int argc, char** argv) {
    if (argc != 8 && argc != 12) {
        fprintf(stderr, "usage: %s L Nt beta kappa form in.bin out.bin [U eps n_md u]\n", argv[0]);
        return 1;
    }
    const int traj = argc == 12;
    hub_params prm = {0};
    prm.L = atoi(argv[1]);
    prm.Nt = atoi(argv[2]);
    prm.beta = atof(argv[3]);
    prm.kappa = atof(argv[4]);
    prm.nrhs_max = 1;
    prm.path = HUB_PATH_AUTO;
    prm.mu = 0.0;
    prm.form = atoi(argv[5]);
    const size_t N = (size_t)2 * prm.L * prm.L * prm.Nt;

    double* phi = malloc(N * sizeof(double));
    double* chi = malloc(2 * N * sizeof(double));
    double* out = malloc(6 * N * sizeof(double));
    double* pi0 = malloc(N * sizeof(double));
    if (!phi || !chi || !out || !pi0) return 1;
    FILE* f = fopen(argv[6], "rb");
    if (!f || fread(phi, sizeof(double), N, f) != N || fread(chi, sizeof(double), 2 * N, f) != 2 * N ||
        (traj && fread(pi0, sizeof(double), N, f) != N)) {
        fprintf(stderr, "cannot read %s\n", argv[6]);
        return 1;
    }
    fclose(f);

    hipStream_t st;
    CHECK_HIP(hipStreamCreate(&st));
    double *d_phi, *d_chi, *d_mv, *d_x, *d_g;
    CHECK_HIP(hipMalloc((void**)&d_phi, N * sizeof(double)));
    CHECK_HIP(hipMalloc((void**)&d_chi, 2 * N * sizeof(double)));
    CHECK_HIP(hipMalloc((void**)&d_mv, 2 * N * sizeof(double)));
    CHECK_HIP(hipMalloc((void**)&d_x, 2 * N * sizeof(double)));
    CHECK_HIP(hipMalloc((void**)&d_g, N * sizeof(double)));
    CHECK_HIP(hipMemcpy(d_phi, phi, N * sizeof(double), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_chi, chi, 2 * N * sizeof(double), hipMemcpyHostToDevice));

    hub_ctx* ctx = NULL;
    CHECK_HUB(hub_create(&prm, st, &ctx));
    CHECK_HUB(hub_apply_M(ctx, d_phi, d_chi, d_mv, 1, st));
    hub_cg_opts opts = {0};
    opts.tol = 1e-10;
    opts.max_iter = 100000;
    opts.reliable_every = 50;
    opts.prec = HUB_PREC_MIXED;
    opts.use_x0 = 0;
    opts.stall_updates = 0;
    hub_cg_info info;
    CHECK_HUB(hub_cg_solve(ctx, d_phi, d_chi, d_x, 1, &opts, &info, st));
    CHECK_HUB(hub_force(ctx, d_phi, d_x, d_g, 1, st));
    CHECK_HIP(hipStreamSynchronize(st));

    CHECK_HIP(hipMemcpy(out, d_mv, 2 * N * sizeof(double), hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(out + 2 * N, d_x, 2 * N * sizeof(double), hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(out + 4 * N, d_g, N * sizeof(double), hipMemcpyDeviceToHost));
    hub_traj_info tinfo = {0};
    if (traj) {
        double* d_pi;
        CHECK_HIP(hipMalloc((void**)&d_pi, N * sizeof(double)));
        CHECK_HIP(hipMemcpy(d_pi, pi0, N * sizeof(double), hipMemcpyHostToDevice));
        hub_traj_opts to = {0};
        to.U = atof(argv[8]);
        to.eps = atof(argv[9]);
        to.n_md = atoi(argv[10]);
        to.integrator = HUB_MD_LEAPFROG;
        to.cg = opts;
        to.cg.tol = 1e-12;
        CHECK_HUB(hub_trajectory(ctx, d_phi, d_pi, d_chi, 1, atof(argv[11]), &to, &tinfo, st));
        CHECK_HIP(hipMemcpy(out + 5 * N, d_phi, N * sizeof(double), hipMemcpyDeviceToHost));
        CHECK_HIP(hipFree(d_pi));
    }
    hub_destroy(ctx);
    CHECK_HIP(hipFree(d_phi));
    CHECK_HIP(hipFree(d_chi));
    CHECK_HIP(hipFree(d_mv));
    CHECK_HIP(hipFree(d_x));
    CHECK_HIP(hipFree(d_g));
    CHECK_HIP(hipStreamDestroy(st));

    f = fopen(argv[7], "wb");
    if (!f || fwrite(out, sizeof(double), 5 * N, f) != 5 * N ||
        fwrite(&info.iters, sizeof(int32_t), 1, f) != 1 ||
        fwrite(&info.true_rel_res, sizeof(double), 1, f) != 1 ||
        (traj && (fwrite(&tinfo.accepted, sizeof(int32_t), 1, f) != 1 ||
                  fwrite(&tinfo.dH, sizeof(double), 1, f) != 1 ||
                  fwrite(out + 5 * N, sizeof(double), N, f) != N))) {
        fprintf(stderr, "cannot write %s\n", argv[7]);
        return 1;
    }
    fclose(f);
    free(phi);
    free(chi);
    free(out);
    free(pi0);
    return 0;
}
