// The split-FP16 projections for r <= 128 (128-column tiles): the
// deep-pipeline register-staged grouped kernel and the LDS-staged one, in a
// file of their own so that they compile in parallel with the other width.
#include "proj_lds.h"

namespace rpmi {

hipError_t launch_split_group_narrow(const GroupEntry* table, int count, int64_t blocks, const GroupEntry* one,
                                  hipStream_t s) {
    if (blocks <= 0 || (count <= 0 && !one)) return hipSuccess;
    using T = NarrowCfg::Tile;
    if (one)
        hipLaunchKernelGGL((project_split_f16_single_kernel<T, NarrowCfg::Depth, false>), dim3((unsigned)blocks),
                           dim3(T::THREADS), 0, s, one->p);
    else
        hipLaunchKernelGGL((project_split_f16_grouped_kernel<T, NarrowCfg::Depth, false>), dim3((unsigned)blocks),
                           dim3(T::THREADS), 0, s, table, count);
    return hipGetLastError();
}

hipError_t launch_split_group_narrow_lds(const GroupEntry* table, int count, int64_t blocks, int64_t rblocks,
                                         hipStream_t s) {
    if (blocks <= 0 || count <= 0) return hipSuccess;
    if (blocks > 0x7FFFFFFF || rblocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL((project_split_lds_grouped_kernel<NarrowLdsCfg>), dim3((unsigned)blocks),
                       dim3(NarrowLdsCfg::THREADS), 0, s, table, count);
    if (rblocks > 0)
        hipLaunchKernelGGL((split_lds_group_reduce_kernel<NarrowLdsCfg>), dim3((unsigned)rblocks),
                           dim3(NarrowLdsCfg::THREADS), 0, s, table, count);
    return hipGetLastError();
}

int64_t split_group_reduce_blocks(int64_t tiles, bool narrow_lds) {
    return tiles * (narrow_lds ? NarrowLdsCfg::TM * NarrowLdsCfg::TN : WideCfg::TM * WideCfg::TN);
}

}  // namespace rpmi
