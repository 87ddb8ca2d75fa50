// Host-side launchers of the kernels in kernels.hip.
#pragma once
#include <hip/hip_runtime_api.h>

#include "mpixs_dev.h"

namespace mpixs {

hipError_t launch_post(hipStream_t s, uint64_t *p, uint64_t v);
hipError_t launch_wait(hipStream_t s, const WaitArgs &a);
hipError_t launch_signal(hipStream_t s, const SignalArgs &a);
hipError_t launch_copy(hipStream_t s, const CopyArgs &a, int w, int nwg, bool fused);
hipError_t launch_reduce(hipStream_t s, const ReduceArgs &a, int basic, int op, bool vec, int nwg,
                         bool fused);
hipError_t launch_batch(hipStream_t s, const BatchArgs &a, int nwg);
int copy_block_units(bool fused);   // units in one copy chunk (one workgroup pass)
int reduce_threads();

}  // namespace mpixs
