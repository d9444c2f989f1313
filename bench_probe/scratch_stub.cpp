// Replaces the library's static device scratch (csrc/scratch.hip) in the
// counter-collection build of the library: no device variable in the code
// object.  pm_check_noalloc returns an error in that build; every other entry
// point and every kernel is the product's, compiled from the same sources.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace pm {

hipError_t scratch_device(void** ptr) {
    *ptr = nullptr;
    return hipErrorNotSupported;
}

int scratch_partials() { return 0; }

}  // namespace pm
