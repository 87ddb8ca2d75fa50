// Test-only recording stand-in for the HIP runtime and the library's kernel
// launchers, so the library's host code runs on the CPU under AddressSanitizer
// and ThreadSanitizer (never linked into libmpixs.so).
//
// Memory calls work on host memory, with a registry of allocations so that
// the library's buffer checks see device and pinned ranges.  Kernel launches
// are counted and otherwise do nothing, except the device stores the host
// side of the library reads back: host flags (batch arena and eager staging
// recycling) and release words (channel-block recycling) of signal, fused
// copy and wait kernels, which are written at once as if the kernel had run.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "../../paper_2208_13707_amd/csrc/mpixs_launch.h"
#include "../../paper_2208_13707_amd/csrc/runtime.h"

namespace {

struct Alloc {
    size_t size;
    hipMemoryType type;
};

std::mutex g_mu;
std::map<uintptr_t, Alloc> g_allocs;
std::atomic<uint64_t> g_launches{0};

void *take(size_t n, hipMemoryType type) {
    void *p = std::aligned_alloc(256, (n + 255) / 256 * 256 + 256);
    if (!p) return nullptr;
    std::memset(p, 0, n);
    std::lock_guard<std::mutex> g(g_mu);
    g_allocs[uintptr_t(p)] = Alloc{n, type};
    return p;
}

hipError_t give(void *p) {
    if (!p) return hipSuccess;
    {
        std::lock_guard<std::mutex> g(g_mu);
        if (!g_allocs.erase(uintptr_t(p))) return hipErrorInvalidValue;
    }
    std::free(p);
    return hipSuccess;
}

bool find(const void *p, uintptr_t *base, Alloc *a) {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_allocs.upper_bound(uintptr_t(p));
    if (it == g_allocs.begin()) return false;
    --it;
    if (uintptr_t(p) >= it->first + it->second.size) return false;
    *base = it->first;
    *a = it->second;
    return true;
}

struct Obj {
    int dummy = 0;
};

}  // namespace

extern "C" uint64_t hipstub_launches() { return g_launches.load(); }

hipError_t hipMalloc(void **p, size_t n) {
    *p = take(n, hipMemoryTypeDevice);
    return *p ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipFree(void *p) { return give(p); }
hipError_t hipHostMalloc(void **p, size_t n, unsigned) {
    *p = take(n, hipMemoryTypeHost);
    return *p ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipHostFree(void *p) { return give(p); }
hipError_t hipMemset(void *p, int v, size_t n) {
    std::memset(p, v, n);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void *p, int v, size_t n, hipStream_t) { return hipMemset(p, v, n); }
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
    std::memcpy(d, s, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t) {
    return hipMemcpy(d, s, n, k);
}
hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t, int) {
    *v = 100000;
    return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    *s = reinterpret_cast<hipStream_t>(new Obj());
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    delete reinterpret_cast<Obj *>(s);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamQuery(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorUnknown; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
    *g = nullptr;
    return hipErrorUnknown;
}
hipError_t hipEventCreate(hipEvent_t *e) {
    *e = reinterpret_cast<hipEvent_t>(new Obj());
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    delete reinterpret_cast<Obj *>(e);
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
    *ms = 0.0f;
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *, hipGraph_t, void *, char *, size_t) {
    return hipErrorUnknown;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorUnknown; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipPointerGetAttributes(hipPointerAttribute_t *a, const void *p) {
    uintptr_t base;
    Alloc al;
    if (!find(p, &base, &al)) return hipErrorInvalidValue;
    std::memset(a, 0, sizeof(*a));
    a->type = al.type;
    a->devicePointer = const_cast<void *>(p);
    return hipSuccess;
}
hipError_t hipMemGetAddressRange(hipDeviceptr_t *base, size_t *size, hipDeviceptr_t p) {
    uintptr_t b;
    Alloc al;
    if (!find(p, &b, &al)) return hipErrorInvalidValue;
    *base = reinterpret_cast<void *>(b);
    *size = al.size;
    return hipSuccess;
}

namespace mpixs {

namespace {
hipError_t counted() {
    g_launches.fetch_add(1, std::memory_order_relaxed);
    return hipSuccess;
}
uint8_t *g_region = nullptr;
uint64_t g_gen = 0;
std::mutex g_region_mu;
int g_k_wait_rel, g_k_signal;
}  // namespace

hipError_t launch_post(hipStream_t, uint64_t *, uint64_t, DevStream *) { return counted(); }
hipError_t launch_wait(hipStream_t, const WaitArgs &a) {
    // the wait "has passed": its releasing lanes write their release words
    if (a.rel_base)
        for (int l = 0; l < a.n && l < 64; ++l)
            if (a.rel_idx[l])
                __atomic_store_n(&a.rel_base[a.rel_idx[l] - 1], a.target[l], __ATOMIC_RELEASE);
    return counted();
}
hipError_t launch_signal(hipStream_t, const SignalArgs &a) {
    if (a.host_flag) __atomic_store_n(a.host_flag, 1u, __ATOMIC_RELEASE);
    if (a.rel_word) __atomic_store_n(a.rel_word, a.rel_val, __ATOMIC_RELEASE);
    return counted();
}
hipError_t launch_copy(hipStream_t, const CopyArgs &a, int, int, bool fused) {
    // a fused copy's last workgroup writes these after done
    if (fused && a.host_flag) __atomic_store_n(a.host_flag, 1u, __ATOMIC_RELEASE);
    if (fused && a.rel_word) __atomic_store_n(a.rel_word, a.rel_val, __ATOMIC_RELEASE);
    return counted();
}
hipError_t launch_reduce(hipStream_t, const ReduceArgs &, int, int, bool, int, bool) {
    return counted();
}
bool reduce_fixed_ok(int n) { return n == 8 || n == 16 || n == 32 || n == 64; }
int reduce_fixed_units() { return 2; }
hipError_t launch_reduce_fixed(hipStream_t, const ReduceArgs &, int, int, int) { return counted(); }
hipError_t launch_reduce_multi(hipStream_t, const MultiRedArgs &, int, int, int, bool) {
    return counted();
}
int reduce_multi_units(bool nt) { return 256 * (nt ? 2 : 1); }
hipError_t launch_batch(hipStream_t, const BatchArgs &, int) { return counted(); }
bool batch_tile_ok(uint32_t t) { return t == 256 || t == 512 || t == 1024 || t == 2048 || t == 4096; }
hipError_t launch_post_inc(hipStream_t, uint64_t *, DevStream *) { return counted(); }
const void *wait_rel_kernel() { return &g_k_wait_rel; }
const void *signal_kernel() { return &g_k_signal; }
hipError_t launch_wait_rel(hipStream_t, const RelWaitArgs &) { return counted(); }
hipError_t build_batch_graph(hipGraph_t *out, const RelWaitArgs *, const BatchArgs &, int,
                             const SignalArgs &) {
    *out = nullptr;
    return hipErrorUnknown;
}
int copy_block_units(bool fused) { return 256 * (fused ? 4 : 1); }
int reduce_threads() { return 256; }

void static_batch_setup(int) {
    std::lock_guard<std::mutex> g(g_region_mu);
    if (!g_region) hipMalloc(reinterpret_cast<void **>(&g_region), kStaticBatchBytes);
}
int static_batch_region(int, size_t bytes, uint8_t **ptr, uint64_t *gen) {
    std::lock_guard<std::mutex> g(g_region_mu);
    if (!g_region) return MPIXS_ERR_GPU;
    if (bytes > kStaticBatchBytes) return MPIXS_ERR_NOMEM;
    *ptr = g_region;
    *gen = ++g_gen;
    return MPIXS_SUCCESS;
}
bool static_batch_current(int, uint64_t gen) {
    std::lock_guard<std::mutex> g(g_region_mu);
    return gen == g_gen;
}

}  // namespace mpixs
