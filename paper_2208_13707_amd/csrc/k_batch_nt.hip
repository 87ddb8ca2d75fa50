// Nontemporal instances of the batch kernel (groups of at least 64 MiB of
// payload by default), compiled apart from the regular ones.
#include <hip/hip_runtime.h>

#include "k_batch_impl.h"

namespace mpixs {

const void *batch_kernel_streaming(uint32_t tile) { return batch_kernel_nt<true>(tile); }

hipError_t launch_batch_streaming(hipStream_t s, const BatchArgs &a, int nwg) {
    return launch_batch_nt<true>(s, a, nwg);
}

}  // namespace mpixs
