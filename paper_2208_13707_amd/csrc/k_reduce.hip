// Canonical-order reduction kernels of the enqueued allreduce (libmpixs,
// gfx950).
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/mpixs.h"
#include "kernels_common.h"
#include "mpixs_dev.h"
#include "mpixs_launch.h"

namespace mpixs {

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
        if (a.trace && !s_fatal && blockIdx.x == 0 && threadIdx.x == 0)
            trace_ev(a.me, MPIXS_TRACE_MATCH, a.arrive, a.arrive_target);
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
            if (a.done_ptr) {
                st_release(a.done_ptr, a.done_val);
                if (a.trace) trace_ev(a.me, MPIXS_TRACE_DONE, a.done_ptr, a.done_val);
            }
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

// A group's reductions of one type and operator in one launch.  Workgroup b
// serves the last instance whose first_wg <= b, chunk b - first_wg of it:
// RED_THREADS x U vectors (aligned instances; chunk 0 also takes the tail
// elements) or RED_THREADS x U elements, U = 2 in nontemporal launches (the
// large ones) and 1 otherwise.  Same left fold in rank order as k_reduce.
// Instances share no byte, so they need no order.
constexpr int RED_MAX_RANKS = 64;

template <typename T, int OP, bool NT>
__global__ void __launch_bounds__(RED_THREADS) k_reduce_multi(MultiRedArgs a) {
    __shared__ uint32_t s_fatal;
    __shared__ MultiRedDesc s_d;
    __shared__ const void *s_ptr[2 * RED_MAX_RANKS];
    const uint32_t b = blockIdx.x;
    if (threadIdx.x == 0) {
        s_fatal = ld_relaxed32(&a.me->fatal);
        s_d = MultiRedDesc{};   // no instance found: the workgroup does nothing
    }
    __syncthreads();
    // first_wg ascends strictly from 0.  Up to RED_THREADS instances every
    // thread reads one descriptor at once (the table may sit in host memory,
    // where dependent reads each cost a bus round trip); beyond, thread 0
    // bisects.
    if (a.ninst <= RED_THREADS) {
        const uint32_t t = threadIdx.x;
        if (t < a.ninst) {
            const MultiRedDesc d = a.desc[t];
            const uint32_t next = t + 1 < a.ninst ? a.desc[t + 1].first_wg : 0xffffffffu;
            if (d.first_wg <= b && b < next) s_d = d;
        }
    } else if (threadIdx.x == 0) {
        uint32_t lo = 0, hi = a.ninst;   // desc[lo].first_wg <= b < desc[hi].first_wg
        while (hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (a.desc[mid].first_wg <= b) lo = mid;
            else hi = mid;
        }
        s_d = a.desc[lo];
    }
    __syncthreads();
    if (s_fatal) return;
    const MultiRedDesc d = s_d;
    const int n = int(d.n);
    if (threadIdx.x < 2 * d.n) s_ptr[threadIdx.x] = a.ptrs[d.ptr + threadIdx.x];
    __syncthreads();
    // a chunk is U passes of RED_THREADS units; lane k-th unit at
    // c * RED_THREADS * U + k * RED_THREADS + threadIdx.x
    constexpr int U = NT ? 2 : 1;
    constexpr int G = RED_GROUP / U;   // inputs of each pass loaded back to back
    const uint64_t base = (blockIdx.x - d.first_wg) * uint64_t(RED_THREADS * U) + threadIdx.x;
    auto fold_one = [&](uint64_t i) {
        T acc = static_cast<const T *>(s_ptr[0])[i];
        for (int q = 1; q < n; ++q) acc = combine<T, OP>(acc, static_cast<const T *>(s_ptr[q])[i]);
        for (int q = 0; q < n; ++q) static_cast<T *>(const_cast<void *>(s_ptr[n + q]))[i] = acc;
    };
    if (d.vec) {
        constexpr int L = int(16 / sizeof(T));
        using V = T __attribute__((ext_vector_type(L)));
        const uint64_t nvec = d.count / L;
        V acc[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const uint64_t v = base + uint64_t(k) * RED_THREADS;
            if (v < nvec) acc[k] = ld_unit<V, NT>(reinterpret_cast<uint64_t>(static_cast<const V *>(s_ptr[0]) + v));
        }
        for (int q0 = 1; q0 < n; q0 += G) {
            V x[U][G];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const uint64_t v = base + uint64_t(k) * RED_THREADS;
#pragma unroll
                for (int j = 0; j < G; ++j)
                    if (v < nvec && q0 + j < n)
                        x[k][j] = ld_unit<V, NT>(
                            reinterpret_cast<uint64_t>(static_cast<const V *>(s_ptr[q0 + j]) + v));
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const uint64_t v = base + uint64_t(k) * RED_THREADS;
#pragma unroll
                for (int j = 0; j < G; ++j)
                    if (v < nvec && q0 + j < n) {
#pragma unroll
                        for (int l = 0; l < L; ++l) acc[k][l] = combine<T, OP>(acc[k][l], x[k][j][l]);
                    }
            }
        }
        for (int q = 0; q < n; ++q) {
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const uint64_t v = base + uint64_t(k) * RED_THREADS;
                if (v < nvec)
                    st_unit<V, NT>(
                        reinterpret_cast<uint64_t>(static_cast<V *>(const_cast<void *>(s_ptr[n + q])) + v), acc[k]);
            }
        }
        if (blockIdx.x == d.first_wg) {
            const uint64_t i = nvec * L + threadIdx.x;
            if (i < d.count) fold_one(i);
        }
    } else {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const uint64_t i = base + uint64_t(k) * RED_THREADS;
            if (i < d.count) fold_one(i);
        }
    }
}

// ------------------------------------------------------------- launchers
int reduce_threads() { return RED_THREADS; }

template <typename T, bool NT>
static hipError_t reduce_multi_t(hipStream_t s, const MultiRedArgs &a, int op, int nwg) {
    switch (op) {
    case OP_SUM: hipLaunchKernelGGL((k_reduce_multi<T, OP_SUM, NT>), dim3(nwg), dim3(RED_THREADS), 0, s, a); break;
    case OP_PROD: hipLaunchKernelGGL((k_reduce_multi<T, OP_PROD, NT>), dim3(nwg), dim3(RED_THREADS), 0, s, a); break;
    case OP_MIN: hipLaunchKernelGGL((k_reduce_multi<T, OP_MIN, NT>), dim3(nwg), dim3(RED_THREADS), 0, s, a); break;
    default: hipLaunchKernelGGL((k_reduce_multi<T, OP_MAX, NT>), dim3(nwg), dim3(RED_THREADS), 0, s, a); break;
    }
    return hipGetLastError();
}

template <bool NT>
static hipError_t reduce_multi_f(hipStream_t s, const MultiRedArgs &a, int basic, int op, int nwg) {
    switch (basic) {
    case MPIXS_INT32: return reduce_multi_t<int32_t, NT>(s, a, op, nwg);
    case MPIXS_INT64: return reduce_multi_t<int64_t, NT>(s, a, op, nwg);
    case MPIXS_FLOAT32: return reduce_multi_t<float, NT>(s, a, op, nwg);
    default: return reduce_multi_t<double, NT>(s, a, op, nwg);
    }
}

int reduce_multi_units(bool nt) { return RED_THREADS * (nt ? 2 : 1); }

hipError_t launch_reduce_multi(hipStream_t s, const MultiRedArgs &a, int basic, int op, int nwg, bool nt) {
    if (a.ninst == 0 || nwg <= 0) return hipErrorInvalidValue;
    return nt ? reduce_multi_f<true>(s, a, basic, op, nwg) : reduce_multi_f<false>(s, a, basic, op, nwg);
}

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
