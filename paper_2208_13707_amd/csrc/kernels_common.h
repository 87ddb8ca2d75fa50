// Device-side helpers shared by the kernels of libmpixs (gfx950).
//
// Memory ordering.  The eight XCDs of an MI355X each have their own L2, so
// a flag that another stream polls is written with a release store at agent
// scope; pollers read it with relaxed agent-scope loads (which go to the
// coherence point) and issue one acquire fence once it holds.  Data written
// by a multi-workgroup kernel is published either at the kernel boundary
// (followed by a one-thread signal kernel) or, in the small fused kernels,
// by one release per workgroup before a completion ticket, the last
// workgroup publishing the done counter.  Kernel boundaries on one stream
// order everything else.
//
// Waits never run forever: they poll with s_sleep, check the world's abort
// word and give up after a wall-clock timeout, recording the error in the
// stream's block; kernels that find their stream failed skip data movement
// but still publish completion, so every waiter downstream also finishes.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/mpixs.h"
#include "mpixs_dev.h"

namespace mpixs {

// ------------------------------------------------------------ primitives
__device__ __forceinline__ uint64_t ld_acquire(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_release(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t ld_relaxed32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t ld_relaxed64(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void set_first_error(DevStream *s, uint32_t e) {
    uint32_t expected = 0;
    __hip_atomic_compare_exchange_strong(&s->first_error, &expected, e, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void set_fatal(DevStream *s, uint32_t e) {
    uint32_t expected = 0;
    __hip_atomic_compare_exchange_strong(&s->fatal, &expected, e, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    set_first_error(s, e);
}

// Poll until *p >= target.  Returns 0, MPIXS_ERR_ABORTED or MPIXS_ERR_TIMEOUT.
// The polls are relaxed agent-scope loads (they read the coherence point);
// one acquire fence follows success.  An acquire load in every poll would
// invalidate caches on each iteration, under the feet of the kernels that
// run beside the waiting wave.
// One trace event from a stream's kernel: a slot of the world's ring by a
// device-wide counter, then one store of the record.
__device__ __forceinline__ void trace_ev(DevStream *me, uint32_t kind, const void *counter,
                                         uint64_t value) {
    TraceEv *ring = me->trace;
    if (!ring) return;
    const uint64_t i = __hip_atomic_fetch_add(me->trace_head, uint64_t(1), __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    TraceEv e;
    e.ticks = wall_clock64();
    e.kind = kind;
    e.stream = me->slot;
    e.counter = reinterpret_cast<uint64_t>(counter);
    e.value = value;
    ring[i & me->trace_mask] = e;
}

__device__ uint32_t spin_wait(const uint64_t *p, uint64_t target, const WaitCtl &ctl) {
    if (ld_relaxed64(p) >= target) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        return 0;
    }
    const uint64_t t0 = wall_clock64();
    uint32_t it = 0;
    for (;;) {
        __builtin_amdgcn_s_sleep(2);
        if (ld_relaxed64(p) >= target) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return 0;
        }
        if ((++it & 31u) == 0) {
            if (__hip_atomic_load(ctl.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))
                return MPIXS_ERR_ABORTED;
            if (wall_clock64() - t0 > ctl.timeout_ticks) return MPIXS_ERR_TIMEOUT;
        }
    }
}

__device__ __forceinline__ void write_status(void *dst, const StatusVal &v, uint32_t fatal) {
    StatusVal *s = reinterpret_cast<StatusVal *>(dst);
    s->source = v.source;
    s->tag = v.tag;
    s->error = fatal ? int32_t(fatal) : v.error;
    s->source_index = v.source_index;
    s->count_bytes = fatal ? 0 : v.count_bytes;
}

// ------------------------------------------------------------------ maps
template <int W> struct Unit;
template <> struct Unit<1> { using T = uint8_t; };
template <> struct Unit<2> { using T = uint16_t; };
template <> struct Unit<4> { using T = uint32_t; };
template <> struct Unit<8> { using T = uint64_t; };
template <> struct Unit<16> { using T = __attribute__((ext_vector_type(4))) uint32_t; };

// Tail of the fused (small) copy and reduce kernels.  The barrier makes the
// workgroup's stores complete in its XCD's L2; one agent-scope release by
// thread 0 then writes that L2 back before the workgroup draws a ticket, and
// the last workgroup publishes completion.  (A release in every wave costs
// an L2 writeback per wave; large transfers instead end at the kernel
// boundary and a separate signal kernel publishes them.)
__device__ __forceinline__ bool last_workgroup(DevStream *me, uint64_t ticket_last) {
    __syncthreads();
    __shared__ int s_last;
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        s_last = 1;
        if (gridDim.x > 1) {
            const uint64_t t = __hip_atomic_fetch_add(&me->ticket, uint64_t(1), __ATOMIC_ACQ_REL,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            s_last = (t == ticket_last);
        }
    }
    __syncthreads();
    return s_last != 0;
}

// Threads of the copy and batch kernels' workgroups.
constexpr int COPY_THREADS = 256;

template <typename T, bool NT>
__device__ __forceinline__ T ld_unit(uint64_t addr) {
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const T *>(addr));
    else return *reinterpret_cast<const T *>(addr);
}

template <typename T, bool NT>
__device__ __forceinline__ void st_unit(uint64_t addr, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<T *>(addr));
    else *reinterpret_cast<T *>(addr) = v;
}

}  // namespace mpixs
