// Batch kernel template of groups and persistent batches (libmpixs,
// gfx950), instantiated in k_batch.hip (regular loads and stores) and
// k_batch_nt.hip (nontemporal), so the two halves compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/mpixs.h"
#include "kernels_common.h"
#include "mpixs_dev.h"

namespace mpixs {

// ----------------------------------------------------------------- batch
// One kernel for every copy of a group.  Workgroup b runs a contiguous range
// of tiles (balanced: base or base + 1), starting at the (message, tile)
// the host computed for it, and walks the messages in order, copying its
// tiles of each message as one run; the message's
// descriptor is read (host-pinned memory for a one-shot group, device
// memory for a persistent batch) into LDS when the workgroup reaches it.
// A tile is TILE * 16 bytes of one message; the unit size and map kinds of
// that message select the copy loop.
template <int TILE, bool NT, int W, int SK, int DK>
__device__ __forceinline__ void tile_copy(const BatchDesc &d, uint64_t u0, uint64_t u1) {
    using T = typename Unit<W>::T;
    // [u0, u1) is a workgroup's run of consecutive tiles of one message; a
    // tile holds TILE * 16 / W units, K per lane.  A lane issues B loads
    // before its first store (the stores could alias later loads, so the
    // compiler cannot hoist them by itself): all of a tile's units up to 8,
    // and at least 2 sixteen-byte or 4 narrower units, so that a run of
    // small-tile units keeps more than one load per lane in flight (4
    // sixteen-byte units per lane measured 15 % slower on contiguous
    // messages)
    constexpr int K = TILE / COPY_THREADS * (16 / W);
    constexpr int BMIN = W == 16 ? 2 : 4;
    constexpr int B = K > BMIN ? (K < 8 ? K : 8) : BMIN;
    for (uint64_t c0 = u0; c0 < u1; c0 += uint64_t(B) * COPY_THREADS) {
        T v[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const uint64_t u = c0 + threadIdx.x + uint64_t(k) * COPY_THREADS;
            if (u < u1) v[k] = ld_unit<T, NT>(map_addr<SK, W>(d.src, u));
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
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
    for (uint64_t i = 0; i < cnt;) {
        if (tin >= sd.ntiles) {
            ++m;
            tin = 0;
            __syncthreads();
            if (threadIdx.x < DW)
                reinterpret_cast<W16 *>(&sd)[threadIdx.x] =
                    reinterpret_cast<const W16 *>(a.desc + m)[threadIdx.x];
            __syncthreads();
        }
        // this workgroup's remaining tiles of message m, copied as one run
        const uint64_t left = cnt - i;
        const uint64_t k = left < uint64_t(sd.ntiles - tin) ? left : uint64_t(sd.ntiles - tin);
        if (!s_fatal) {
            const uint64_t tu = uint64_t(TILE) * (16u / sd.w);   // units per tile
            const uint64_t u0 = uint64_t(tin) * tu;
            const uint64_t u1 = u0 + k * tu < sd.units ? u0 + k * tu : sd.units;
            if (tin + k == sd.ntiles && threadIdx.x < sd.tail) {
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
        tin += uint32_t(k);
        i += k;
    }
}


template <bool NT>
const void *batch_kernel_nt(uint32_t tile) {
    switch (tile) {
    case 256: return reinterpret_cast<const void *>(&k_batch<256, NT>);
    case 512: return reinterpret_cast<const void *>(&k_batch<512, NT>);
    case 1024: return reinterpret_cast<const void *>(&k_batch<1024, NT>);
    case 2048: return reinterpret_cast<const void *>(&k_batch<2048, NT>);
    case 4096: return reinterpret_cast<const void *>(&k_batch<4096, NT>);
    default: return nullptr;
    }
}

template <bool NT>
hipError_t launch_batch_nt(hipStream_t s, const BatchArgs &a, int nwg) {
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

// the nontemporal instances, defined in k_batch_nt.hip
const void *batch_kernel_streaming(uint32_t tile);
hipError_t launch_batch_streaming(hipStream_t s, const BatchArgs &a, int nwg);

}  // namespace mpixs
