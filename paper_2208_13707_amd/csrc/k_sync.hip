// Stream-ordered flag kernels of libmpixs: post, wait, signal, and the
// relative forms used by persistent batches.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/mpixs.h"
#include "kernels_common.h"
#include "mpixs_dev.h"
#include "mpixs_launch.h"

namespace mpixs {

// ----------------------------------------------------------- post / wait
// "This stream reached this point": one release store (and a POST event
// when `tr`, the stream's block, is given).
__global__ void __launch_bounds__(64) k_post(uint64_t *p, uint64_t v, DevStream *tr) {
    if (threadIdx.x == 0) {
        st_release(p, v);
        if (tr) trace_ev(tr, MPIXS_TRACE_POST, p, v);
    }
}

// Lane q waits for *ptr[q] >= target[q]; then lane 0 writes the optional
// status and the stream's first error.
__global__ void __launch_bounds__(64) k_wait(WaitArgs a) {
    const int lane = threadIdx.x;
    uint32_t err = 0;
    const uint32_t fatal0 = ld_relaxed32(&a.me->fatal);
    if (!fatal0 && lane < a.n) {
        err = spin_wait(a.ptr[lane], a.target[lane], a.ctl);
        if (!err && a.trace) trace_ev(a.me, a.trace, a.ptr[lane], a.target[lane]);
        // after spin_wait's acquire fence: nothing of this message touches
        // the block any more, so the host may hand it on
        if (!err && a.rel_base && a.rel_idx[lane])
            __hip_atomic_store(a.rel_base + (a.rel_idx[lane] - 1), a.target[lane],
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (err) set_fatal(a.me, err);
    __syncthreads();
    if (lane == 0) {
        const uint32_t fatal = ld_relaxed32(&a.me->fatal);
        if (a.status) write_status(a.status, a.st, fatal);
        if (!fatal && a.st.error) set_first_error(a.me, uint32_t(a.st.error));
    }
}

// Completion after a data kernel of the same stream: the kernel boundary
// already made its stores visible at agent scope, so one release store
// publishes them.
__global__ void __launch_bounds__(64) k_signal(SignalArgs a) {
    if (threadIdx.x != 0) return;
    const uint32_t fatal = ld_relaxed32(&a.me->fatal);
    if (a.status) write_status(a.status, a.st, fatal);
    if (!fatal && a.set_error && a.st.error) set_first_error(a.me, uint32_t(a.st.error));
    if (a.done_ptr) {
        const uint64_t v = a.inc ? ld_acquire(a.done_ptr) + 1 : a.done_val;
        st_release(a.done_ptr, v);
        if (a.trace) trace_ev(a.me, MPIXS_TRACE_DONE, a.done_ptr, v);
    }
    if (a.host_flag) __hip_atomic_store(a.host_flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    // release: done lands before the host may hand the block to a new owner
    if (a.rel_word) __hip_atomic_store(a.rel_word, a.rel_val, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Persistent batches keep their counters relative: each run of a rank adds
// one to its own arrive counter, and waits compare against counters read on
// the device, so the launch arguments never change between runs.
__global__ void __launch_bounds__(64) k_post_inc(uint64_t *p, DevStream *tr) {
    if (threadIdx.x == 0) {
        const uint64_t v = ld_acquire(p) + 1;
        st_release(p, v);
        if (tr) trace_ev(tr, MPIXS_TRACE_POST, p, v);
    }
}

__global__ void __launch_bounds__(64) k_wait_rel(RelWaitArgs a) {
    const uint32_t lane = threadIdx.x;
    uint32_t err = 0;
    const uint32_t fatal0 = ld_relaxed32(&a.me->fatal);
    if (!fatal0 && lane < a.n && !((a.skip >> lane) & 1u)) {
        const uint64_t target = ld_acquire(a.base) + a.delta;
        err = spin_wait(a.ptr0 + uint64_t(lane) * a.stride, target, a.ctl);
        if (!err && a.trace) trace_ev(a.me, a.trace, a.ptr0 + uint64_t(lane) * a.stride, target);
    }
    if (err) set_fatal(a.me, err);
}

// ------------------------------------------------------------- launchers
hipError_t launch_post_inc(hipStream_t s, uint64_t *p, DevStream *tr) {
    hipLaunchKernelGGL(k_post_inc, dim3(1), dim3(64), 0, s, p, tr);
    return hipGetLastError();
}

hipError_t launch_wait_rel(hipStream_t s, const RelWaitArgs &a) {
    hipLaunchKernelGGL(k_wait_rel, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_post(hipStream_t s, uint64_t *p, uint64_t v, DevStream *tr) {
    hipLaunchKernelGGL(k_post, dim3(1), dim3(64), 0, s, p, v, tr);
    return hipGetLastError();
}

hipError_t launch_wait(hipStream_t s, const WaitArgs &a) {
    hipLaunchKernelGGL(k_wait, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_signal(hipStream_t s, const SignalArgs &a) {
    hipLaunchKernelGGL(k_signal, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

const void *wait_rel_kernel() { return reinterpret_cast<const void *>(&k_wait_rel); }
const void *signal_kernel() { return reinterpret_cast<const void *>(&k_signal); }

}  // namespace mpixs
