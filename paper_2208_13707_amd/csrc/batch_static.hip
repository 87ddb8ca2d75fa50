// Device memory for persistent batches planned without an allocation
// (mpixs_group_end_init_static): a file-scope array of fixed size, of which
// every GPU the library runs on holds its own copy until the process ends.
//
// In host code the array's name is a host-side stand-in, not a device
// address.  Its address on a device is asked for once per device, with that
// device current, when the first world on it is created, and only that
// address is ever handed to kernels or copies.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "../../include/mpixs.h"
#include "runtime.h"

namespace mpixs {

static __device__ __align__(256) uint8_t scratch[kStaticBatchBytes];

namespace {

struct DeviceScratch {
    uint8_t *ptr = nullptr;     // this device's copy of scratch
    hipError_t err = hipSuccess;
    uint64_t gen = 0;           // static plans written to it so far
};

std::mutex g_mu;
std::map<int, DeviceScratch> g_dev;

}  // namespace

void static_batch_setup(int device) {
    std::lock_guard<std::mutex> g(g_mu);
    if (g_dev.count(device)) return;
    DeviceScratch d;
    void *p = nullptr;
    d.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (d.err != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    d.ptr = static_cast<uint8_t *>(p);
    g_dev[device] = d;
}

int static_batch_region(int device, size_t bytes, uint8_t **ptr, uint64_t *gen) {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_dev.find(device);
    if (it == g_dev.end() || !it->second.ptr) return MPIXS_ERR_GPU;
    if (bytes > kStaticBatchBytes) return MPIXS_ERR_NOMEM;
    *ptr = it->second.ptr;
    *gen = ++it->second.gen;
    return MPIXS_SUCCESS;
}

bool static_batch_current(int device, uint64_t gen) {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_dev.find(device);
    return it != g_dev.end() && it->second.gen == gen;
}

}  // namespace mpixs
