// The deep-pipeline split-FP16 projection for r > 128 (256-column tiles):
// one instantiation of the grouped kernel, in a file of its own so that it
// compiles in parallel with the other width.
#include "proj_common.h"

namespace rpmi {

hipError_t launch_split_group_wide(const GroupArgs& ga, hipStream_t s) {
    const int64_t blocks = ga.start[ga.count];
    if (blocks <= 0) return hipSuccess;
    using T = WideCfg::Tile;
    hipLaunchKernelGGL((project_split_f16_grouped_kernel<T, WideCfg::Depth, kDmaTwoAcc>), dim3((unsigned)blocks),
                       dim3(T::THREADS), 0, s, ga);
    return hipGetLastError();
}

}  // namespace rpmi
