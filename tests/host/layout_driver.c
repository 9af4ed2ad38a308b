/* Prints sizeof/offsetof of the ABI structs as the C compiler lays them out. */
#include <stddef.h>
#include <stdio.h>

#include "hub.h"

int main(void) {
    printf("hub_params %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(hub_params), offsetof(hub_params, L),
           offsetof(hub_params, Nt), offsetof(hub_params, beta), offsetof(hub_params, kappa),
           offsetof(hub_params, nrhs_max), offsetof(hub_params, path), offsetof(hub_params, mu),
           offsetof(hub_params, form));
    printf("hub_cg_opts %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(hub_cg_opts), offsetof(hub_cg_opts, tol),
           offsetof(hub_cg_opts, max_iter), offsetof(hub_cg_opts, reliable_every), offsetof(hub_cg_opts, prec),
           offsetof(hub_cg_opts, use_x0), offsetof(hub_cg_opts, stall_updates), offsetof(hub_cg_opts, history_host),
           offsetof(hub_cg_opts, history_len));
    printf("hub_cg_info %zu %zu %zu %zu %zu %zu\n", sizeof(hub_cg_info), offsetof(hub_cg_info, iters),
           offsetof(hub_cg_info, reliable_updates), offsetof(hub_cg_info, true_rel_res),
           offsetof(hub_cg_info, recursive_rel_res), offsetof(hub_cg_info, persistent_launches));
    printf("hub_traj_opts %zu %zu %zu %zu %zu %zu\n", sizeof(hub_traj_opts), offsetof(hub_traj_opts, U),
           offsetof(hub_traj_opts, eps), offsetof(hub_traj_opts, n_md), offsetof(hub_traj_opts, integrator),
           offsetof(hub_traj_opts, cg));
    printf("hub_traj_info %zu %zu %zu %zu %zu %zu %zu\n", sizeof(hub_traj_info), offsetof(hub_traj_info, accepted),
           offsetof(hub_traj_info, n_forces), offsetof(hub_traj_info, cg_iters), offsetof(hub_traj_info, H0),
           offsetof(hub_traj_info, H1), offsetof(hub_traj_info, dH));
    return 0;
}
