// Device scratch of rp_project_packed_noalloc(): a file-scope device array
// that holds the contraction-split partial sums and arrival counters of the
// split-FP16 projection, so that the entry point allocates nothing.  Each
// device that loads the library holds its own copy until the process ends.
// Host code never uses the array's name as an address: the device address
// comes from hipGetSymbolAddress(), taken once per device when a context is
// created with that device current.
#include "rpmi_internal.h"

namespace rpmi {

__device__ __align__(256) unsigned char scratch[kNoAllocPartialBytes + kNoAllocCounterBytes];

hipError_t noalloc_scratch_address(void** out) {
    *out = nullptr;
    return hipGetSymbolAddress(out, HIP_SYMBOL(scratch));
}

}  // namespace rpmi
