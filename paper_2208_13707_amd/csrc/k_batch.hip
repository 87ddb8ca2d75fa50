// Batch kernel of groups and persistent batches (libmpixs, gfx950): the
// regular-access instances, the launch dispatch and the graph of a
// persistent run.
#include <hip/hip_runtime.h>

#include <cstring>

#include "k_batch_impl.h"
#include "mpixs_launch.h"

namespace mpixs {

// ------------------------------------------------------------- launchers
static const void *batch_kernel(uint32_t tile, bool nt) {
    return nt ? batch_kernel_streaming(tile) : batch_kernel_nt<false>(tile);
}

bool batch_tile_ok(uint32_t tile) { return batch_kernel(tile, false) != nullptr; }

hipError_t launch_batch(hipStream_t s, const BatchArgs &a, int nwg) {
    return a.nt ? launch_batch_streaming(s, a, nwg) : launch_batch_nt<false>(s, a, nwg);
}

// The leader's part of one run of a persistent batch as a graph: [relative
// wait for every other rank's arrival] -> batch kernel -> signal (done + 1).
// Kernel node arguments are copied when the nodes are added.
hipError_t build_batch_graph(hipGraph_t *out, const RelWaitArgs *w, const BatchArgs &a, int nwg,
                             const SignalArgs &sg) {
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    hipGraphNode_t prev = nullptr, node = nullptr;
    hipKernelNodeParams p;
    if (w) {
        RelWaitArgs wa = *w;
        void *args[] = {&wa};
        std::memset(&p, 0, sizeof(p));
        p.func = const_cast<void *>(wait_rel_kernel());
        p.gridDim = dim3(1);
        p.blockDim = dim3(64);
        p.kernelParams = args;
        e = hipGraphAddKernelNode(&node, g, nullptr, 0, &p);
        if (e != hipSuccess) { (void)hipGraphDestroy(g); return e; }
        prev = node;
    }
    BatchArgs ba = a;
    void *args[] = {&ba};
    std::memset(&p, 0, sizeof(p));
    p.func = const_cast<void *>(batch_kernel(a.tile, a.nt != 0));
    if (!p.func || nwg < 1) { (void)hipGraphDestroy(g); return hipErrorInvalidValue; }
    p.gridDim = dim3(unsigned(nwg));
    p.blockDim = dim3(COPY_THREADS);
    p.kernelParams = args;
    e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); return e; }
    prev = node;
    SignalArgs sa = sg;
    void *sargs[] = {&sa};
    std::memset(&p, 0, sizeof(p));
    p.func = const_cast<void *>(signal_kernel());
    p.gridDim = dim3(1);
    p.blockDim = dim3(64);
    p.kernelParams = sargs;
    e = hipGraphAddKernelNode(&node, g, &prev, 1, &p);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); return e; }
    *out = g;
    return hipSuccess;
}

}  // namespace mpixs
