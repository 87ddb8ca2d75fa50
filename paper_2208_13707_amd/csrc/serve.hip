// Open-loop request server over the enqueue path (see include/mpixs_driver.h).
//
// A harness: every message and reduction of a request goes through the
// public enqueue calls; the kernels here only make payloads (fill), check
// results (checksum) and report completion to the host.
#include <hip/hip_runtime.h>

#include <immintrin.h>
#include <linux/futex.h>
#include <sys/syscall.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/mpixs_driver.h"

namespace {

using clk = std::chrono::steady_clock;

// ------------------------------------------------------------------ kernels
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Byte j = byte (j mod 8) of splitmix64(seed * 2^32 + j / 8).
__global__ void __launch_bounds__(256) k_fill(uint8_t *p, int64_t n, uint64_t seed) {
    const int64_t words = (n + 7) / 8;
    for (int64_t w = int64_t(blockIdx.x) * 256 + threadIdx.x; w < words;
         w += int64_t(gridDim.x) * 256) {
        const uint64_t v = splitmix64((seed << 32) + uint64_t(w));
        if (8 * w + 8 <= n && (reinterpret_cast<uintptr_t>(p) & 7) == 0) {
            reinterpret_cast<uint64_t *>(p)[w] = v;
        } else {
            for (int b = 0; b < 8 && 8 * w + b < n; ++b) p[8 * w + b] = uint8_t(v >> (8 * b));
        }
    }
}

// weight * sum_j byte_j * (j + 1) mod 2^64, accumulated with device atomics
// in acc[0]; the last of `total` workgroups (of this launch and of the other
// launches into the same accumulator; ticket in acc[1]) publishes the sum
// and the completion flag to host memory.
__global__ void __launch_bounds__(256) k_checksum(const uint8_t *p, int64_t n, uint64_t weight,
                                                   uint64_t total, uint64_t *acc,
                                                   uint64_t *host_sum, uint32_t *host_flag) {
    uint64_t s = 0;
    for (int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x; j < n; j += int64_t(gridDim.x) * 256)
        s += uint64_t(p[j]) * uint64_t(j + 1);
    __shared__ uint64_t red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < unsigned(o)) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    __hip_atomic_fetch_add(&acc[0], red[0] * weight, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t t = __hip_atomic_fetch_add(&acc[1], uint64_t(1), __ATOMIC_ACQ_REL,
                                              __HIP_MEMORY_SCOPE_AGENT);
    if (t + 1 != total) return;
    *host_sum = __hip_atomic_load(&acc[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(host_flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

int grid_for(int64_t n, int64_t per_thread) {
    const int64_t g = (n + 256 * per_thread - 1) / (256 * per_thread);
    return int(std::max<int64_t>(1, std::min<int64_t>(g, 1024)));
}

// ------------------------------------------------------------ device arena
// First-fit allocator over one device allocation of the budget.
class Arena {
  public:
    explicit Arena(size_t cap) : cap_(cap) { free_[0] = cap; }
    // blocks until `n` bytes fit; false on timeout, once `stop` is set, or if
    // n exceeds the budget
    bool alloc(size_t n, size_t *off, std::chrono::milliseconds timeout,
               const std::atomic<int> &stop) {
        std::unique_lock<std::mutex> g(mu_);
        if (n > cap_) return false;
        const auto until = clk::now() + timeout;
        for (;;) {
            if (stop.load()) return false;
            for (auto it = free_.begin(); it != free_.end(); ++it) {
                if (it->second >= n) {
                    *off = it->first;
                    const size_t rest = it->second - n;
                    const size_t at = it->first + n;
                    free_.erase(it);
                    if (rest) free_[at] = rest;
                    return true;
                }
            }
            if (clk::now() >= until) return false;
            cv_.wait_for(g, std::chrono::milliseconds(10));
        }
    }
    void release(size_t off, size_t n) {
        {
            std::lock_guard<std::mutex> g(mu_);
            auto it = free_.emplace(off, n).first;
            auto nx = std::next(it);
            if (nx != free_.end() && it->first + it->second == nx->first) {
                it->second += nx->second;
                free_.erase(nx);
            }
            if (it != free_.begin()) {
                auto pv = std::prev(it);
                if (pv->first + pv->second == it->first) {
                    pv->second += it->second;
                    free_.erase(it);
                }
            }
        }
        cv_.notify_all();
    }

  private:
    size_t cap_;
    std::map<size_t, size_t> free_;
    std::mutex mu_;
    std::condition_variable cv_;
};

struct Slot {
    std::atomic<uint32_t> admitted{0};
    size_t off = 0, bytes = 0;
};

// 64 rank threads share the host's cores, so threads that wait for another
// thread sleep on a futex word (bounded to 1 ms, so a failure elsewhere is
// always noticed) instead of spinning.
void futex_wait(std::atomic<uint32_t> &w, uint32_t seen) {
    struct timespec ts = {0, 1000000};
    syscall(SYS_futex, reinterpret_cast<uint32_t *>(&w), FUTEX_WAIT_PRIVATE, seen, &ts, nullptr, 0);
}

void futex_wake(std::atomic<uint32_t> &w) {
    syscall(SYS_futex, reinterpret_cast<uint32_t *>(&w), FUTEX_WAKE_PRIVATE, INT32_MAX, nullptr,
            nullptr, 0);
}

size_t round256(int64_t n) { return size_t((n + 255) / 256 * 256); }

}  // namespace

extern "C" int mpixs_drv_serve(mpixs_world world, int nranks, const mpixs_comm *comms,
                               void *const *streams, const mpixs_drv_req *reqs, int64_t nreq,
                               int64_t budget_bytes, mpixs_drv_req_result *results,
                               double *wall_s, const int64_t *capture, int64_t ncapture,
                               void *capture_dev, int flags) {
    const bool mode = (flags & MPIXS_DRV_SERVE_HOST_SYNCED) != 0;
    const bool rank0_sum = (flags & MPIXS_DRV_SERVE_RANK0_SUM) != 0;
    if (!world || nranks <= 0 || !comms || !streams || nreq < 0 || nreq >= INT32_MAX ||
        (nreq > 0 && (!reqs || !results)) ||
        (flags & ~(MPIXS_DRV_SERVE_HOST_SYNCED | MPIXS_DRV_SERVE_RANK0_SUM)) ||
        budget_bytes <= 0 || ncapture < 0 || (ncapture > 0 && (!capture || !capture_dev)))
        return MPIXS_ERR_ARG;
    std::vector<int64_t> cap_off(size_t(std::max<int64_t>(nreq, 0)), -1);
    for (int64_t k = 0; k < ncapture; ++k) {
        if (capture[2 * k] < 0 || capture[2 * k] >= nreq || capture[2 * k + 1] < 0)
            return MPIXS_ERR_ARG;
        cap_off[size_t(capture[2 * k])] = capture[2 * k + 1];
    }
    for (int64_t i = 0; i < nreq; ++i) {
        const mpixs_drv_req &q = reqs[i];
        const bool p2p = q.kind == MPIXS_DRV_REQ_SENDRECV || q.kind == MPIXS_DRV_REQ_ISEND_WAIT;
        if ((!p2p && q.kind != MPIXS_DRV_REQ_ALLREDUCE) || q.bytes < 0 || q.bytes > INT32_MAX ||
            (i > 0 && q.arrival_us < reqs[i - 1].arrival_us) ||
            (p2p && (q.src < 0 || q.src >= nranks || q.dst < 0 || q.dst >= nranks ||
                     q.src == q.dst)) ||
            (!p2p && q.bytes % 4))
            return MPIXS_ERR_ARG;
    }
    char *arena_mem = nullptr;
    uint64_t *dsum = nullptr;
    uint64_t *hsum = nullptr;
    uint32_t *hflag = nullptr;
    const size_t nslot = size_t(std::max<int64_t>(nreq, 1));
    if (hipMalloc(reinterpret_cast<void **>(&arena_mem), size_t(budget_bytes)) != hipSuccess)
        return MPIXS_ERR_NOMEM;
    if (hipMalloc(reinterpret_cast<void **>(&dsum), nslot * 16) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&hsum), nslot * 8, hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&hflag), nslot * 4, hipHostMallocCoherent) !=
            hipSuccess) {
        (void)hipFree(arena_mem);
        if (dsum) (void)hipFree(dsum);
        if (hsum) (void)hipHostFree(hsum);
        return MPIXS_ERR_NOMEM;
    }
    (void)hipMemset(dsum, 0, nslot * 16);
    (void)hipDeviceSynchronize();
    std::memset(hsum, 0, nslot * 8);
    std::memset(hflag, 0, nslot * 4);

    Arena arena{static_cast<size_t>(budget_bytes)};
    std::vector<Slot> slots(static_cast<size_t>(nslot));
    std::vector<std::vector<int64_t>> mine(static_cast<size_t>(nranks));
    for (int64_t i = 0; i < nreq; ++i) {
        const mpixs_drv_req &q = reqs[i];
        std::memset(&results[i], 0, sizeof(results[i]));
        if (q.kind == MPIXS_DRV_REQ_ALLREDUCE) {
            for (int r = 0; r < nranks; ++r) mine[size_t(r)].push_back(i);
        } else {
            mine[size_t(q.src)].push_back(i);
            if (q.dst != q.src) mine[size_t(q.dst)].push_back(i);
        }
    }
    std::mutex admit_mu;
    std::deque<int64_t> admitted;          // admission order, for the reaper
    std::atomic<int64_t> completed{0};
    std::atomic<int> first_error{0};
    std::atomic<int> go{0};
    clk::time_point t0;
    auto us_since = [&](clk::time_point t) {
        return std::chrono::duration<double, std::micro>(t - t0).count();
    };
    auto fail = [&](int rc) {
        int z = 0;
        first_error.compare_exchange_strong(z, rc);
        mpixs_world_abort(world);
    };

    // Admission (one thread): first come, first served in arrival order,
    // each request as soon as it has arrived and its buffers fit into the
    // arena.  The admitted requests are then always a prefix of the
    // schedule, and a rank thread only ever waits for an earlier request, so
    // memory can never fill up with requests that depend on one still
    // waiting for memory; and admission never waits for a busy rank thread.
    auto admitter = [&]() {
        while (!go.load(std::memory_order_acquire)) _mm_pause();
        for (int64_t i = 0; i < nreq && !first_error.load(); ++i) {
            const mpixs_drv_req &q = reqs[i];
            const auto arrive = t0 + std::chrono::duration_cast<clk::duration>(
                                         std::chrono::duration<double, std::micro>(q.arrival_us));
            if (arrive - clk::now() > std::chrono::microseconds(200))
                std::this_thread::sleep_until(arrive - std::chrono::microseconds(100));
            while (clk::now() < arrive) _mm_pause();
            const size_t each = round256(q.bytes);
            const size_t need = q.kind == MPIXS_DRV_REQ_ALLREDUCE ? 2 * each * size_t(nranks)
                                                                  : 2 * each;
            size_t off = 0;
            if (!arena.alloc(need, &off, std::chrono::milliseconds(60000), first_error)) {
                results[i].error = MPIXS_ERR_NOMEM;
                fail(MPIXS_ERR_NOMEM);
                break;
            }
            Slot &sl = slots[size_t(i)];
            sl.off = off;
            sl.bytes = need;
            results[i].admit_us = us_since(clk::now());
            {
                std::lock_guard<std::mutex> g(admit_mu);
                admitted.push_back(i);
            }
            sl.admitted.store(1, std::memory_order_release);
            futex_wake(sl.admitted);
        }
    };

    auto worker = [&](int r) {
        hipStream_t hs = static_cast<hipStream_t>(streams[r]);
        mpixs_comm c = comms[r];
        while (!go.load(std::memory_order_acquire)) _mm_pause();
        for (int64_t i : mine[size_t(r)]) {
            if (first_error.load()) break;
            const mpixs_drv_req &q = reqs[i];
            Slot &sl = slots[size_t(i)];
            for (int spin = 0; !sl.admitted.load(std::memory_order_acquire); ++spin) {
                if (first_error.load()) return;
                if (spin < 64) _mm_pause();
                else futex_wait(sl.admitted, 0);
            }
            const size_t each = round256(q.bytes);
            char *base = arena_mem + sl.off;
            int rc = MPIXS_SUCCESS;
            if (q.kind == MPIXS_DRV_REQ_ALLREDUCE) {
                uint8_t *in = reinterpret_cast<uint8_t *>(base + each * size_t(r));
                uint8_t *out = reinterpret_cast<uint8_t *>(base + each * size_t(nranks + r));
                hipLaunchKernelGGL(k_fill, dim3(grid_for(q.bytes, 8)), dim3(256), 0, hs, in,
                                   q.bytes, q.seed + uint64_t(r));
                rc = mode ? mpixs_allreduce(in, out, int(q.bytes / 4), MPIXS_INT32, MPIXS_SUM, c)
                          : mpixs_allreduce_enqueue(in, out, int(q.bytes / 4), MPIXS_INT32, MPIXS_SUM,
                                                    c);
                if (!rc && cap_off[size_t(i)] >= 0 &&
                    hipMemcpyAsync(static_cast<char *>(capture_dev) + cap_off[size_t(i)] +
                                       size_t(r) * size_t(q.bytes),
                                   out, size_t(q.bytes), hipMemcpyDeviceToDevice, hs) != hipSuccess)
                    rc = MPIXS_ERR_GPU;
                if (!rc && (!rank0_sum || r == 0)) {
                    // every rank checksums its own output (or rank 0 alone);
                    // the last workgroup of the launches publishes the sum
                    const int g = grid_for(q.bytes, 64);
                    const uint64_t parts = rank0_sum ? 1 : uint64_t(nranks);
                    hipLaunchKernelGGL(k_checksum, dim3(g), dim3(256), 0, hs, out, q.bytes,
                                       rank0_sum ? uint64_t(1) : uint64_t(2 * r + 1),
                                       uint64_t(g) * parts, dsum + 2 * i, hsum + i, hflag + i);
                }
            } else {
                uint8_t *sb = reinterpret_cast<uint8_t *>(base);
                uint8_t *rb = reinterpret_cast<uint8_t *>(base + each);
                const int tag = q.kind;
                if (r == q.src) {
                    hipLaunchKernelGGL(k_fill, dim3(grid_for(q.bytes, 8)), dim3(256), 0, hs, sb,
                                       q.bytes, q.seed);
                    if (mode) {
                        rc = mpixs_send(sb, int(q.bytes), MPIXS_UINT8, q.dst, tag, c);
                    } else if (q.kind == MPIXS_DRV_REQ_SENDRECV) {
                        rc = mpixs_send_enqueue(sb, int(q.bytes), MPIXS_UINT8, q.dst, tag, c);
                    } else {
                        mpixs_request rq = nullptr;
                        rc = mpixs_isend_enqueue(sb, int(q.bytes), MPIXS_UINT8, q.dst, tag, c, &rq);
                        if (!rc) rc = mpixs_wait_enqueue(&rq, nullptr);
                    }
                }
                if (!rc && r == q.dst) {
                    if (mode) {
                        rc = mpixs_recv(rb, int(q.bytes), MPIXS_UINT8, q.src, tag, c, nullptr);
                    } else if (q.kind == MPIXS_DRV_REQ_SENDRECV) {
                        rc = mpixs_recv_enqueue(rb, int(q.bytes), MPIXS_UINT8, q.src, tag, c,
                                                nullptr);
                    } else {
                        mpixs_request rq = nullptr;
                        rc = mpixs_irecv_enqueue(rb, int(q.bytes), MPIXS_UINT8, q.src, tag, c, &rq);
                        if (!rc) rc = mpixs_wait_enqueue(&rq, nullptr);
                    }
                    if (!rc && cap_off[size_t(i)] >= 0 &&
                        hipMemcpyAsync(static_cast<char *>(capture_dev) + cap_off[size_t(i)], rb,
                                       size_t(q.bytes), hipMemcpyDeviceToDevice,
                                       hs) != hipSuccess)
                        rc = MPIXS_ERR_GPU;
                    if (!rc) {
                        const int g = grid_for(q.bytes, 64);
                        hipLaunchKernelGGL(k_checksum, dim3(g), dim3(256), 0, hs, rb, q.bytes,
                                           uint64_t(1), uint64_t(g), dsum + 2 * i, hsum + i,
                                           hflag + i);
                    }
                }
            }
            if (rc) {
                results[i].error = rc;
                fail(rc);
                break;
            }
        }
    };

    // reaper: completion flags in admission order are not required; scan all
    // outstanding admitted requests
    auto reaper = [&]() {
        std::vector<int64_t> live;
        while (completed.load() < nreq) {
            {
                std::lock_guard<std::mutex> g(admit_mu);
                while (!admitted.empty()) {
                    live.push_back(admitted.front());
                    admitted.pop_front();
                }
            }
            bool any = false;
            for (size_t k = 0; k < live.size();) {
                const int64_t i = live[k];
                if (__atomic_load_n(&hflag[i], __ATOMIC_ACQUIRE)) {
                    results[i].done_us = us_since(clk::now());
                    results[i].checksum = hsum[i];
                    arena.release(slots[size_t(i)].off, slots[size_t(i)].bytes);
                    completed.fetch_add(1);
                    live[k] = live.back();
                    live.pop_back();
                    any = true;
                } else {
                    ++k;
                }
            }
            if (first_error.load() && live.empty()) break;
            if (!any) std::this_thread::yield();
        }
    };

    std::vector<std::thread> th;
    for (int r = 0; r < nranks; ++r) th.emplace_back(worker, r);
    std::thread ad(admitter);
    t0 = clk::now();
    go.store(1, std::memory_order_release);
    std::thread rp(reaper);
    ad.join();
    for (auto &x : th) x.join();
    // requests that failed before completing will never set their flag
    if (first_error.load()) {
        mpixs_world_wait(world, 60000);
        completed.store(nreq);
    }
    rp.join();
    double last = 0;
    for (int64_t i = 0; i < nreq; ++i) last = std::max(last, results[i].done_us);
    if (wall_s) *wall_s = last * 1e-6;
    (void)hipDeviceSynchronize();
    (void)hipFree(arena_mem);
    (void)hipFree(dsum);
    (void)hipHostFree(hsum);
    (void)hipHostFree(hflag);
    return first_error.load();
}
