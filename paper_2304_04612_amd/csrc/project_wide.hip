// The LDS-staged split-FP16 projection for r > 128 (256-column tiles): the
// grouped (exact split) and single (folded split) forms, in a file of their
// own so that they compile in parallel with the other width.
#include "proj_lds.h"

namespace rpmi {

hipError_t launch_split_group_wide(const GroupEntry* table, int count, int64_t blocks, const GroupEntry* one,
                                   hipStream_t s, int64_t rblocks) {
    if (blocks <= 0 || (count <= 0 && !one)) return hipSuccess;
    using C = WideCfg;
    if (one) {
        hipLaunchKernelGGL((project_split_lds_single_kernel<C>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s,
                           one->p);
        if (one->p.ksplit > 1) {
            const int64_t tiles = one->tiles_m * one->tiles_n;
            hipLaunchKernelGGL((split_lds_reduce_kernel<C>), dim3((unsigned)(tiles * C::TM * C::TN)), dim3(C::THREADS),
                               0, s, one->p);
        }
    }
    else {
        hipLaunchKernelGGL((project_split_lds_grouped_kernel<C>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s,
                           table, count);
        if (rblocks > 0)
            hipLaunchKernelGGL((split_lds_group_reduce_kernel<C>), dim3((unsigned)rblocks), dim3(C::THREADS), 0, s,
                               table, count);
    }
    return hipGetLastError();
}

}  // namespace rpmi
