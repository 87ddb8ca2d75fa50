// Typemap-driven copy kernel of one matched message (libmpixs, gfx950).
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/mpixs.h"
#include "kernels_common.h"
#include "mpixs_dev.h"
#include "mpixs_launch.h"

namespace mpixs {

// ------------------------------------------------------------------ copy
// Unit u of the packed message goes from map_src(u) to map_dst(u); W is the
// largest power of two (<= 16) that divides every block boundary and base
// address of both sides, so each unit is one aligned load and one store.
// Workgroups take chunks of COPY_THREADS * U consecutive units; within a
// chunk lane i handles units i, i + 256, ... so every load and store
// instruction of a wave covers consecutive units.
//
// FUSED: small messages, at most kFusedMaxWG workgroups that loop over the
// chunks with U = 4 units per lane in flight.  Thread 0 of every workgroup
// first waits for the other side's ready counter, and the last workgroup
// publishes completion.
// Otherwise (large messages): one chunk of 256 units per workgroup, one
// unit per lane, streaming (nontemporal) loads and stores -- the fastest
// shape measured on gfx950 -- and nothing else: the stream waited before the
// kernel and a k_signal follows it.
constexpr int COPY_UNROLL_FUSED = 4;


template <int W, int SK, int DK, bool FUSED>
__global__ void __launch_bounds__(COPY_THREADS) k_copy(CopyArgs a) {
    using T = typename Unit<W>::T;
    constexpr int COPY_UNROLL = FUSED ? COPY_UNROLL_FUSED : 1;
    constexpr bool NT = !FUSED;
    __shared__ uint32_t s_fatal;
    if (threadIdx.x == 0) {
        uint32_t f = ld_relaxed32(&a.me->fatal);
        if (FUSED && !f && a.wait_ptr) {
            f = spin_wait(a.wait_ptr, a.wait_target, a.ctl);
            if (f) set_fatal(a.me, f);
        }
        s_fatal = f;
    }
    __syncthreads();
    if (FUSED && a.wait_ptr) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (FUSED && a.trace && a.wait_ptr && !s_fatal && blockIdx.x == 0 && threadIdx.x == 0)
        trace_ev(a.me, MPIXS_TRACE_MATCH, a.wait_ptr, a.wait_target);
    if (!s_fatal) {
        const uint64_t n = a.units;
        constexpr uint64_t CH = uint64_t(COPY_THREADS) * COPY_UNROLL;
        const uint64_t nch = (n + CH - 1) / CH;
        for (uint64_t c = blockIdx.x; c < nch; c += gridDim.x) {
            const uint64_t b = c * CH + threadIdx.x;
            T v[COPY_UNROLL];
#pragma unroll
            for (int k = 0; k < COPY_UNROLL; ++k) {
                const uint64_t u = b + uint64_t(k) * COPY_THREADS;
                if (u < n) v[k] = ld_unit<T, NT>(map_addr<SK, W>(a.src, u));
            }
#pragma unroll
            for (int k = 0; k < COPY_UNROLL; ++k) {
                const uint64_t u = b + uint64_t(k) * COPY_THREADS;
                if (u < n) st_unit<T, NT>(map_addr<DK, W>(a.dst, u), v[k]);
            }
        }
    }
    if constexpr (FUSED) {
        if (last_workgroup(a.me, a.ticket_last) && threadIdx.x == 0) {
            const uint32_t fatal = ld_relaxed32(&a.me->fatal);
            if (a.status) write_status(a.status, a.st, fatal);
            if (!fatal && a.set_error && a.st.error) set_first_error(a.me, uint32_t(a.st.error));
            if (a.done_ptr) {
                st_release(a.done_ptr, a.done_val);
                if (a.trace) trace_ev(a.me, MPIXS_TRACE_DONE, a.done_ptr, a.done_val);
            }
            if (a.host_flag)
                __hip_atomic_store(a.host_flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            // release: the done store above lands before the host may hand
            // the block to a new owner
            if (a.rel_word)
                __hip_atomic_store(a.rel_word, a.rel_val, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// ------------------------------------------------------------- launchers
int copy_block_units(bool fused) { return COPY_THREADS * (fused ? COPY_UNROLL_FUSED : 1); }

template <int W, int SK, bool F>
static hipError_t copy_dk(hipStream_t s, const CopyArgs &a, int dk, int nwg) {
    switch (dk) {
    case MAP_CONTIG: hipLaunchKernelGGL((k_copy<W, SK, MAP_CONTIG, F>), dim3(nwg), dim3(COPY_THREADS), 0, s, a); break;
    case MAP_VEC: hipLaunchKernelGGL((k_copy<W, SK, MAP_VEC, F>), dim3(nwg), dim3(COPY_THREADS), 0, s, a); break;
    default: hipLaunchKernelGGL((k_copy<W, SK, MAP_SEG, F>), dim3(nwg), dim3(COPY_THREADS), 0, s, a); break;
    }
    return hipGetLastError();
}

template <int W, bool F>
static hipError_t copy_w(hipStream_t s, const CopyArgs &a, int nwg) {
    switch (a.src.kind) {
    case MAP_CONTIG: return copy_dk<W, MAP_CONTIG, F>(s, a, a.dst.kind, nwg);
    case MAP_VEC: return copy_dk<W, MAP_VEC, F>(s, a, a.dst.kind, nwg);
    default: return copy_dk<W, MAP_SEG, F>(s, a, a.dst.kind, nwg);
    }
}

template <bool F>
static hipError_t copy_f(hipStream_t s, const CopyArgs &a, int w, int nwg) {
    switch (w) {
    case 16: return copy_w<16, F>(s, a, nwg);
    case 8: return copy_w<8, F>(s, a, nwg);
    case 4: return copy_w<4, F>(s, a, nwg);
    case 2: return copy_w<2, F>(s, a, nwg);
    default: return copy_w<1, F>(s, a, nwg);
    }
}

hipError_t launch_copy(hipStream_t s, const CopyArgs &a, int w, int nwg, bool fused) {
    return fused ? copy_f<true>(s, a, w, nwg) : copy_f<false>(s, a, w, nwg);
}

}  // namespace mpixs
