/* Prints sizeof/offsetof of the public structs as the C compiler lays them out. */
#include <stddef.h>
#include <stdio.h>

#include "../../include/hjr.h"

#define F(T, m) printf("%s.%s %zu\n", #T, #m, offsetof(T, m))
int main(void)
{
    printf("hjr_grid %zu\nhjr_dynamics %zu\nhjr_options %zu\nhjr_result %zu\nhjr_problem %zu\nhjr_ctx_stats %zu\n",
           sizeof(hjr_grid), sizeof(hjr_dynamics), sizeof(hjr_options), sizeof(hjr_result), sizeof(hjr_problem),
           sizeof(hjr_ctx_stats));
    printf("hjr_kernel_time %zu\nhjr_profile %zu\n", sizeof(hjr_kernel_time), sizeof(hjr_profile));
    F(hjr_kernel_time, ms); F(hjr_kernel_time, working_launches); F(hjr_kernel_time, working_ms);
    F(hjr_profile, stage64);
    F(hjr_grid, lo); F(hjr_grid, periodic_mask);
    F(hjr_options, cfl); F(hjr_options, max_iter); F(hjr_options, stall_window); F(hjr_options, brs); F(hjr_options, discount); F(hjr_options, local_updates);
    F(hjr_result, seconds); F(hjr_result, converged); F(hjr_result, discounted_iterations); F(hjr_result, node_updates);
    F(hjr_problem, opts); F(hjr_problem, l); F(hjr_problem, result); F(hjr_problem, status);
    return 0;
}
