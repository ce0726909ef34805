// The deep-pipeline split-FP16 projection for r <= 128 (128-column tiles):
// one instantiation of the grouped kernel, in a file of its own so that it
// compiles in parallel with the other width.
#include "proj_common.h"

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

}  // namespace rpmi
