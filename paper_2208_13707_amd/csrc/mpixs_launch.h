// Host-side launchers of the kernels (k_sync.hip, k_copy.hip, k_reduce.hip,
// k_batch.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include "mpixs_dev.h"

namespace mpixs {

hipError_t launch_post(hipStream_t s, uint64_t *p, uint64_t v, DevStream *tr);   // tr: POST event (nullptr: none)
hipError_t launch_wait(hipStream_t s, const WaitArgs &a);
hipError_t launch_signal(hipStream_t s, const SignalArgs &a);
hipError_t launch_copy(hipStream_t s, const CopyArgs &a, int w, int nwg, bool fused);
hipError_t launch_reduce(hipStream_t s, const ReduceArgs &a, int basic, int op, bool vec, int nwg,
                         bool fused);
// large reductions over 8, 16, 32 or 64 ranks with 16-byte aligned buffers
bool reduce_fixed_ok(int n);
int reduce_fixed_units();            // vectors per lane of launch_reduce_fixed
hipError_t launch_reduce_fixed(hipStream_t s, const ReduceArgs &a, int basic, int op, int nwg);
// a group's reductions of one type and operator, one workgroup per chunk of
// reduce_multi_units(nt) vectors (or elements when not 16-byte aligned); nt:
// nontemporal vector loads and stores (launches much larger than the caches)
hipError_t launch_reduce_multi(hipStream_t s, const MultiRedArgs &a, int basic, int op, int nwg, bool nt);
int reduce_multi_units(bool nt);     // vectors (or elements) per workgroup of launch_reduce_multi
hipError_t launch_batch(hipStream_t s, const BatchArgs &a, int nwg);
bool batch_tile_ok(uint32_t tile);   // a tile size the batch kernel is built for
hipError_t launch_post_inc(hipStream_t s, uint64_t *p, DevStream *tr);
const void *wait_rel_kernel();        // kernel handles for graph nodes
const void *signal_kernel();
hipError_t launch_wait_rel(hipStream_t s, const RelWaitArgs &a);
// leader's run of a persistent batch: [wait] -> batch -> signal (w may be null)
hipError_t build_batch_graph(hipGraph_t *out, const RelWaitArgs *w, const BatchArgs &a, int nwg,
                             const SignalArgs &sg);
int copy_block_units(bool fused);   // units in one copy chunk (one workgroup pass)
int reduce_threads();

}  // namespace mpixs
