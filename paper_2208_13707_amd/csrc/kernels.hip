// CDNA4 (gfx950) kernels of libmpixs: stream-ordered flags, typemap-driven
// copy of a matched message, and the canonical-order allreduce.
//
// Memory ordering.  The eight XCDs of an MI355X each have their own L2, so
// a flag that another stream polls is written with a release store at agent
// scope and read with acquire loads at agent scope; data written by a
// multi-workgroup kernel is released by every wave before the workgroup
// draws a completion ticket, and only the last workgroup publishes the done
// counter.  Kernel boundaries on one stream order everything else.
//
// Waits never run forever: they poll with s_sleep, check the world's abort
// word and give up after a wall-clock timeout, recording the error in the
// stream's block; kernels that find their stream failed skip data movement
// but still publish completion, so every waiter downstream also finishes.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/mpixs.h"
#include "mpixs_dev.h"
#include "mpixs_launch.h"

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
    s->reserved = 0;
    s->count_bytes = fatal ? 0 : v.count_bytes;
}

// ----------------------------------------------------------- post / wait
// "This stream reached this point": one release store.
__global__ void __launch_bounds__(64) k_post(uint64_t *p, uint64_t v) {
    if (threadIdx.x == 0) st_release(p, v);
}

// Lane q waits for *ptr[q] >= target[q]; then lane 0 writes the optional
// status and the stream's first error.
__global__ void __launch_bounds__(64) k_wait(WaitArgs a) {
    const int lane = threadIdx.x;
    uint32_t err = 0;
    const uint32_t fatal0 = ld_relaxed32(&a.me->fatal);
    if (!fatal0 && lane < a.n) err = spin_wait(a.ptr[lane], a.target[lane], a.ctl);
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
    if (a.done_ptr) st_release(a.done_ptr, a.inc ? ld_acquire(a.done_ptr) + 1 : a.done_val);
    if (a.host_flag) __hip_atomic_store(a.host_flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Persistent batches keep their counters relative: each run of a rank adds
// one to its own arrive counter, and waits compare against counters read on
// the device, so the launch arguments never change between runs.
__global__ void __launch_bounds__(64) k_post_inc(uint64_t *p) {
    if (threadIdx.x == 0) st_release(p, ld_acquire(p) + 1);
}

__global__ void __launch_bounds__(64) k_wait_rel(RelWaitArgs a) {
    const uint32_t lane = threadIdx.x;
    uint32_t err = 0;
    const uint32_t fatal0 = ld_relaxed32(&a.me->fatal);
    if (!fatal0 && lane < a.n && !((a.skip >> lane) & 1u)) {
        const uint64_t target = ld_acquire(a.base) + a.delta;
        err = spin_wait(a.ptr0 + uint64_t(lane) * a.stride, target, a.ctl);
    }
    if (err) set_fatal(a.me, err);
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
constexpr int COPY_THREADS = 256;
constexpr int COPY_UNROLL_FUSED = 4;

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
            if (a.done_ptr) st_release(a.done_ptr, a.done_val);
        }
    }
}

// ---------------------------------------------------------------- reduce
template <typename T> struct Uns { using U = T; };
template <> struct Uns<int32_t> { using U = uint32_t; };
template <> struct Uns<int64_t> { using U = uint64_t; };

template <typename T, int OP>
__device__ __forceinline__ T combine(T acc, T x) {
    if constexpr (OP == OP_SUM) {
        using U = typename Uns<T>::U;
        return T(U(acc) + U(x));
    } else if constexpr (OP == OP_PROD) {
        using U = typename Uns<T>::U;
        return T(U(acc) * U(x));
    } else if constexpr (OP == OP_MIN) {
        return x < acc ? x : acc;
    } else {
        return x > acc ? x : acc;
    }
}

constexpr int RED_THREADS = 256;
constexpr int RED_GROUP = 16;   // inputs loaded back to back before folding

// out_q[i] = (((in_0[i] op in_1[i]) op in_2[i]) ... op in_{n-1}[i]) for every q:
// the left fold in rank order, each element owned by one lane (16 bytes of
// elements per lane when every buffer is 16-byte aligned).  Workgroups take
// chunks of RED_THREADS vectors.  FUSED: small collectives; threads q < n
// of every workgroup wait for rank q's arrive counter first and the last
// workgroup publishes done.
template <typename T, int OP, bool VEC, bool FUSED>
__global__ void __launch_bounds__(RED_THREADS) k_reduce(ReduceArgs a) {
    __shared__ uint32_t s_fatal;
    if (threadIdx.x == 0) s_fatal = ld_relaxed32(&a.me->fatal);
    __syncthreads();
    if (FUSED && a.arrive && !s_fatal) {
        uint32_t err = 0;
        const int q = threadIdx.x;
        if (q < a.n && q != a.me_rank) err = spin_wait(a.arrive + q * 16, a.arrive_target, a.ctl);
        if (err) set_fatal(a.me, err);
        __syncthreads();
        if (threadIdx.x == 0) s_fatal = ld_relaxed32(&a.me->fatal);
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    if (!s_fatal) {
        const int n = a.n;
        constexpr int L = VEC ? int(16 / sizeof(T)) : 1;
        using V = T __attribute__((ext_vector_type(L)));
        const uint64_t nvec = a.count / L;
        const uint64_t nch = (nvec + RED_THREADS - 1) / RED_THREADS;
        for (uint64_t c = blockIdx.x; c < nch; c += gridDim.x) {
            const uint64_t v = c * RED_THREADS + threadIdx.x;
            if (v < nvec) {
                constexpr bool NT = !FUSED;
                V acc = ld_unit<V, NT>(reinterpret_cast<uint64_t>(reinterpret_cast<const V *>(a.in[0]) + v));
                for (int q0 = 1; q0 < n; q0 += RED_GROUP) {
                    V x[RED_GROUP];
#pragma unroll
                    for (int j = 0; j < RED_GROUP; ++j)
                        if (q0 + j < n)
                            x[j] = ld_unit<V, NT>(
                                reinterpret_cast<uint64_t>(reinterpret_cast<const V *>(a.in[q0 + j]) + v));
#pragma unroll
                    for (int j = 0; j < RED_GROUP; ++j)
                        if (q0 + j < n) {
#pragma unroll
                            for (int l = 0; l < L; ++l) acc[l] = combine<T, OP>(acc[l], x[j][l]);
                        }
                }
                for (int q = 0; q < n; ++q)
                    st_unit<V, NT>(reinterpret_cast<uint64_t>(reinterpret_cast<V *>(a.out[q]) + v), acc);
            }
        }
        if constexpr (VEC) {
            // tail elements that do not fill a vector
            const uint64_t gtid = uint64_t(blockIdx.x) * RED_THREADS + threadIdx.x;
            const uint64_t i = nvec * L + gtid;
            if (i < a.count) {
                T acc = reinterpret_cast<const T *>(a.in[0])[i];
                for (int q = 1; q < n; ++q)
                    acc = combine<T, OP>(acc, reinterpret_cast<const T *>(a.in[q])[i]);
                for (int q = 0; q < n; ++q) reinterpret_cast<T *>(a.out[q])[i] = acc;
            }
        }
    }
    if constexpr (FUSED) {
        if (last_workgroup(a.me, a.ticket_last) && threadIdx.x == 0) {
            if (a.done_ptr) st_release(a.done_ptr, a.done_val);
        }
    }
}

// Large reductions over a rank count known at compile time (8, 16, 32 or
// 64, 16-byte aligned buffers): each lane folds RED_FIXED_U vectors, and
// with the inputs unrolled the loads of all ranks are in flight together
// (measured about 7 % faster than the runtime-n loop at 16 x 64 MiB).  Same
// canonical order: acc = in_0, then acc = acc (+) in_q for q = 1 .. N-1.
constexpr int RED_FIXED_U = 2;

template <typename T, int OP, int N>
__global__ void __launch_bounds__(RED_THREADS) k_reduce_n(ReduceArgs a) {
    __shared__ uint32_t s_fatal;
    if (threadIdx.x == 0) s_fatal = ld_relaxed32(&a.me->fatal);
    __syncthreads();
    if (s_fatal) return;
    constexpr int L = int(16 / sizeof(T));
    constexpr int U = RED_FIXED_U;
    using V = T __attribute__((ext_vector_type(L)));
    const uint64_t nvec = a.count / L;
    constexpr uint64_t CH = uint64_t(RED_THREADS) * U;
    const uint64_t nch = (nvec + CH - 1) / CH;
    for (uint64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        V acc[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const uint64_t v = c * CH + threadIdx.x + uint64_t(k) * RED_THREADS;
            if (v < nvec)
                acc[k] = ld_unit<V, true>(reinterpret_cast<uint64_t>(reinterpret_cast<const V *>(a.in[0]) + v));
        }
#pragma unroll
        for (int q = 1; q < N; ++q) {
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const uint64_t v = c * CH + threadIdx.x + uint64_t(k) * RED_THREADS;
                if (v < nvec) {
                    const V x = ld_unit<V, true>(
                        reinterpret_cast<uint64_t>(reinterpret_cast<const V *>(a.in[q]) + v));
#pragma unroll
                    for (int l = 0; l < L; ++l) acc[k][l] = combine<T, OP>(acc[k][l], x[l]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < N; ++q) {
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const uint64_t v = c * CH + threadIdx.x + uint64_t(k) * RED_THREADS;
                if (v < nvec)
                    st_unit<V, true>(reinterpret_cast<uint64_t>(reinterpret_cast<V *>(a.out[q]) + v), acc[k]);
            }
        }
    }
    // tail elements that do not fill a vector
    const uint64_t gtid = uint64_t(blockIdx.x) * RED_THREADS + threadIdx.x;
    const uint64_t i = nvec * L + gtid;
    if (i < a.count) {
        T acc = reinterpret_cast<const T *>(a.in[0])[i];
        for (int q = 1; q < N; ++q) acc = combine<T, OP>(acc, reinterpret_cast<const T *>(a.in[q])[i]);
        for (int q = 0; q < N; ++q) reinterpret_cast<T *>(a.out[q])[i] = acc;
    }
}

// ----------------------------------------------------------------- batch
// One kernel for every copy of a group.  Workgroup b runs a contiguous range
// of tiles (balanced: base or base + 1), starting at the (message, tile)
// the host computed for it, and walks the messages in order; the message's
// descriptor is read from host-pinned memory into LDS when the workgroup
// reaches it.  A tile is up to BATCH_TILE units of one message; the unit
// size and map kinds of that message select the copy loop.
template <int TILE, bool NT, int W, int SK, int DK>
__device__ __forceinline__ void tile_copy(const BatchDesc &d, uint64_t u0, uint64_t u1) {
    using T = typename Unit<W>::T;
    constexpr int U = TILE / COPY_THREADS;
    // a tile of TILE * 16 bytes is 16 / W chunks of TILE units
    for (uint64_t c0 = u0; c0 < u1; c0 += TILE) {
        T v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const uint64_t u = c0 + threadIdx.x + uint64_t(k) * COPY_THREADS;
            if (u < u1) v[k] = ld_unit<T, NT>(map_addr<SK, W>(d.src, u));
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const uint64_t u = c0 + threadIdx.x + uint64_t(k) * COPY_THREADS;
            if (u < u1) st_unit<T, NT>(map_addr<DK, W>(d.dst, u), v[k]);
        }
    }
}

template <int TILE, bool NT, int W, int SK>
__device__ __forceinline__ void tile_copy_dk(const BatchDesc &d, uint64_t u0, uint64_t u1) {
    switch (d.dst.kind) {
    case MAP_CONTIG: tile_copy<TILE, NT, W, SK, MAP_CONTIG>(d, u0, u1); break;
    case MAP_VEC: tile_copy<TILE, NT, W, SK, MAP_VEC>(d, u0, u1); break;
    default: tile_copy<TILE, NT, W, SK, MAP_SEG>(d, u0, u1); break;
    }
}

template <int TILE, bool NT, int W>
__device__ __forceinline__ void tile_copy_w(const BatchDesc &d, uint64_t u0, uint64_t u1) {
    switch (d.src.kind) {
    case MAP_CONTIG: tile_copy_dk<TILE, NT, W, MAP_CONTIG>(d, u0, u1); break;
    case MAP_VEC: tile_copy_dk<TILE, NT, W, MAP_VEC>(d, u0, u1); break;
    default: tile_copy_dk<TILE, NT, W, MAP_SEG>(d, u0, u1); break;
    }
}

// NT: nontemporal loads and stores (groups much larger than the caches)
template <int TILE, bool NT>
__global__ void __launch_bounds__(COPY_THREADS) k_batch(BatchArgs a) {
    __shared__ BatchDesc sd;
    __shared__ uint32_t s_fatal;
    // descriptors live in host memory: lanes fetch one 16-byte word each so a
    // descriptor costs one round trip over the fabric
    constexpr int DW = sizeof(BatchDesc) / 16;
    using W16 = __attribute__((ext_vector_type(4))) uint32_t;
    const uint32_t b = blockIdx.x;
    const uint64_t cnt = a.nmsg ? a.base + (b < a.extra ? 1 : 0) : 0;
    uint32_t m = cnt ? a.start[b].msg : 0;
    uint32_t tin = cnt ? a.start[b].tile : 0;
    if (threadIdx.x == 0) s_fatal = ld_relaxed32(&a.me->fatal);
    if (cnt && threadIdx.x < DW)
        reinterpret_cast<W16 *>(&sd)[threadIdx.x] =
            reinterpret_cast<const W16 *>(a.desc + m)[threadIdx.x];
    __syncthreads();
    for (uint64_t i = 0; i < cnt; ++i) {
        if (tin >= sd.ntiles) {
            ++m;
            tin = 0;
            __syncthreads();
            if (threadIdx.x < DW)
                reinterpret_cast<W16 *>(&sd)[threadIdx.x] =
                    reinterpret_cast<const W16 *>(a.desc + m)[threadIdx.x];
            __syncthreads();
        }
        if (!s_fatal) {
            const uint64_t tu = uint64_t(TILE) * (16u / sd.w);   // units per tile
            const uint64_t u0 = uint64_t(tin) * tu;
            const uint64_t u1 = u0 + tu < sd.units ? u0 + tu : sd.units;
            if (tin + 1 == sd.ntiles && threadIdx.x < sd.tail) {
                // byte tail of a copy dense on both sides
                const uint64_t off = sd.units * sd.w + threadIdx.x;
                reinterpret_cast<uint8_t *>(sd.dst.base)[off] =
                    reinterpret_cast<const uint8_t *>(sd.src.base)[off];
            }
            if (u0 < u1) {
                switch (sd.w) {
                case 16: tile_copy_w<TILE, NT, 16>(sd, u0, u1); break;
                case 8: tile_copy_w<TILE, NT, 8>(sd, u0, u1); break;
                case 4: tile_copy_w<TILE, NT, 4>(sd, u0, u1); break;
                case 2: tile_copy_w<TILE, NT, 2>(sd, u0, u1); break;
                default: tile_copy_w<TILE, NT, 1>(sd, u0, u1); break;
                }
            }
        }
        if (tin == 0 && threadIdx.x == 0) {
            if (sd.status) write_status(sd.status, sd.st, s_fatal);
            if (!s_fatal && sd.st.error && sd.rstream)
                set_first_error(sd.rstream, uint32_t(sd.st.error));
        }
        ++tin;
    }
}

// ------------------------------------------------------------- launchers
template <bool NT>
static const void *batch_kernel_nt(uint32_t tile) {
    switch (tile) {
    case 256: return reinterpret_cast<const void *>(&k_batch<256, NT>);
    case 512: return reinterpret_cast<const void *>(&k_batch<512, NT>);
    case 1024: return reinterpret_cast<const void *>(&k_batch<1024, NT>);
    case 2048: return reinterpret_cast<const void *>(&k_batch<2048, NT>);
    case 4096: return reinterpret_cast<const void *>(&k_batch<4096, NT>);
    default: return nullptr;
    }
}

static const void *batch_kernel(uint32_t tile, bool nt) {
    return nt ? batch_kernel_nt<true>(tile) : batch_kernel_nt<false>(tile);
}

bool batch_tile_ok(uint32_t tile) { return batch_kernel(tile, false) != nullptr; }

template <bool NT>
static hipError_t launch_batch_nt(hipStream_t s, const BatchArgs &a, int nwg) {
    switch (a.tile) {
    case 256: hipLaunchKernelGGL((k_batch<256, NT>), dim3(nwg), dim3(COPY_THREADS), 0, s, a); break;
    case 512: hipLaunchKernelGGL((k_batch<512, NT>), dim3(nwg), dim3(COPY_THREADS), 0, s, a); break;
    case 1024: hipLaunchKernelGGL((k_batch<1024, NT>), dim3(nwg), dim3(COPY_THREADS), 0, s, a); break;
    case 2048: hipLaunchKernelGGL((k_batch<2048, NT>), dim3(nwg), dim3(COPY_THREADS), 0, s, a); break;
    case 4096: hipLaunchKernelGGL((k_batch<4096, NT>), dim3(nwg), dim3(COPY_THREADS), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch(hipStream_t s, const BatchArgs &a, int nwg) {
    return a.nt ? launch_batch_nt<true>(s, a, nwg) : launch_batch_nt<false>(s, a, nwg);
}

hipError_t launch_post_inc(hipStream_t s, uint64_t *p) {
    hipLaunchKernelGGL(k_post_inc, dim3(1), dim3(64), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_wait_rel(hipStream_t s, const RelWaitArgs &a) {
    hipLaunchKernelGGL(k_wait_rel, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
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
        p.func = const_cast<void *>(reinterpret_cast<const void *>(&k_wait_rel));
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
    p.func = const_cast<void *>(reinterpret_cast<const void *>(&k_signal));
    p.gridDim = dim3(1);
    p.blockDim = dim3(64);
    p.kernelParams = sargs;
    e = hipGraphAddKernelNode(&node, g, &prev, 1, &p);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); return e; }
    *out = g;
    return hipSuccess;
}

hipError_t launch_post(hipStream_t s, uint64_t *p, uint64_t v) {
    hipLaunchKernelGGL(k_post, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_wait(hipStream_t s, const WaitArgs &a) {
    hipLaunchKernelGGL(k_wait, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

int copy_block_units(bool fused) { return COPY_THREADS * (fused ? COPY_UNROLL_FUSED : 1); }

hipError_t launch_signal(hipStream_t s, const SignalArgs &a) {
    hipLaunchKernelGGL(k_signal, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

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

int reduce_threads() { return RED_THREADS; }

template <typename T, int OP, bool F>
static hipError_t reduce_op(hipStream_t s, const ReduceArgs &a, bool vec, int nwg) {
    if (vec) hipLaunchKernelGGL((k_reduce<T, OP, true, F>), dim3(nwg), dim3(RED_THREADS), 0, s, a);
    else hipLaunchKernelGGL((k_reduce<T, OP, false, F>), dim3(nwg), dim3(RED_THREADS), 0, s, a);
    return hipGetLastError();
}

template <typename T, bool F>
static hipError_t reduce_t(hipStream_t s, const ReduceArgs &a, int op, bool vec, int nwg) {
    switch (op) {
    case OP_SUM: return reduce_op<T, OP_SUM, F>(s, a, vec, nwg);
    case OP_PROD: return reduce_op<T, OP_PROD, F>(s, a, vec, nwg);
    case OP_MIN: return reduce_op<T, OP_MIN, F>(s, a, vec, nwg);
    default: return reduce_op<T, OP_MAX, F>(s, a, vec, nwg);
    }
}

template <bool F>
static hipError_t reduce_f(hipStream_t s, const ReduceArgs &a, int basic, int op, bool vec,
                           int nwg) {
    switch (basic) {
    case MPIXS_INT32: return reduce_t<int32_t, F>(s, a, op, vec, nwg);
    case MPIXS_INT64: return reduce_t<int64_t, F>(s, a, op, vec, nwg);
    case MPIXS_FLOAT32: return reduce_t<float, F>(s, a, op, vec, nwg);
    default: return reduce_t<double, F>(s, a, op, vec, nwg);
    }
}

hipError_t launch_reduce(hipStream_t s, const ReduceArgs &a, int basic, int op, bool vec, int nwg,
                         bool fused) {
    return fused ? reduce_f<true>(s, a, basic, op, vec, nwg) : reduce_f<false>(s, a, basic, op, vec, nwg);
}

bool reduce_fixed_ok(int n) { return n == 8 || n == 16 || n == 32 || n == 64; }
int reduce_fixed_units() { return RED_FIXED_U; }

template <typename T, int OP>
static hipError_t reduce_fixed_n(hipStream_t s, const ReduceArgs &a, int nwg) {
    switch (a.n) {
    case 8: hipLaunchKernelGGL((k_reduce_n<T, OP, 8>), dim3(nwg), dim3(RED_THREADS), 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_reduce_n<T, OP, 16>), dim3(nwg), dim3(RED_THREADS), 0, s, a); break;
    case 32: hipLaunchKernelGGL((k_reduce_n<T, OP, 32>), dim3(nwg), dim3(RED_THREADS), 0, s, a); break;
    case 64: hipLaunchKernelGGL((k_reduce_n<T, OP, 64>), dim3(nwg), dim3(RED_THREADS), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t reduce_fixed_t(hipStream_t s, const ReduceArgs &a, int op, int nwg) {
    switch (op) {
    case OP_SUM: return reduce_fixed_n<T, OP_SUM>(s, a, nwg);
    case OP_PROD: return reduce_fixed_n<T, OP_PROD>(s, a, nwg);
    case OP_MIN: return reduce_fixed_n<T, OP_MIN>(s, a, nwg);
    default: return reduce_fixed_n<T, OP_MAX>(s, a, nwg);
    }
}

hipError_t launch_reduce_fixed(hipStream_t s, const ReduceArgs &a, int basic, int op, int nwg) {
    switch (basic) {
    case MPIXS_INT32: return reduce_fixed_t<int32_t>(s, a, op, nwg);
    case MPIXS_INT64: return reduce_fixed_t<int64_t>(s, a, op, nwg);
    case MPIXS_FLOAT32: return reduce_fixed_t<float>(s, a, op, nwg);
    default: return reduce_fixed_t<double>(s, a, op, nwg);
    }
}

}  // namespace mpixs
