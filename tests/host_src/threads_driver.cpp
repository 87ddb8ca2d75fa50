// Threaded patterns of the library's host side, run against the recording
// HIP stand-in (hipstub.cpp) under AddressSanitizer or ThreadSanitizer (large
// groups whose waiting ranks help plan them among them):
// every call's return code is checked, nothing moves data.  Patterns: a
// 32-rank uneven batch through the plain enqueue path, 16-rank enqueued
// allreduces, one-shot groups with allreduces, persistent batches, ordered-
// queue matching with wildcard receives from racing senders, the
// host-synchronised calls, stream and communicator create/free cycles with
// block recycling, a 64-block matching table, datatypes made and freed from
// every thread, and a static (no-allocation) persistent plan.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mpixs.h"

extern "C" uint64_t hipstub_launches();

namespace {

std::atomic<int> g_fail{0};

#define CHECK(expr)                                                                    \
    do {                                                                               \
        const int rc_ = (expr);                                                        \
        if (rc_ != MPIXS_SUCCESS) {                                                    \
            std::fprintf(stderr, "%s:%d: %s -> %s\n", __FILE__, __LINE__, #expr,       \
                         mpixs_error_string(rc_));                                     \
            g_fail.store(1);                                                           \
            return;                                                                    \
        }                                                                              \
    } while (0)

#define EXPECT(cond)                                                                   \
    do {                                                                               \
        if (!(cond)) {                                                                 \
            std::fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond);   \
            g_fail.store(1);                                                           \
            return;                                                                    \
        }                                                                              \
    } while (0)

void run_threads(int n, const std::function<void(int)> &f) {
    std::vector<std::thread> th;
    for (int r = 0; r < n; ++r) th.emplace_back(f, r);
    for (auto &t : th) t.join();
}

struct Rank {
    hipStream_t hs = nullptr;
    mpixs_stream st = nullptr;
    mpixs_comm comm = nullptr;
};

// every rank: a HIP stream, an mpixs stream and a stream communicator
std::vector<Rank> setup(mpixs_world w, int n) {
    std::vector<Rank> R(static_cast<size_t>(n));
    run_threads(n, [&](int r) {
        hipStreamCreateWithFlags(&R[size_t(r)].hs, hipStreamNonBlocking);
        mpixs_info info;
        CHECK(mpixs_info_create(&info));
        CHECK(mpixs_info_set(info, "type", "hipStream_t"));
        CHECK(mpixs_info_set_hex(info, "value", &R[size_t(r)].hs, sizeof(hipStream_t)));
        CHECK(mpixs_stream_create(w, info, &R[size_t(r)].st));
        CHECK(mpixs_info_free(&info));
        mpixs_comm wc;
        CHECK(mpixs_world_comm(w, r, &wc));
        CHECK(mpixs_comm_create_with_stream(wc, R[size_t(r)].st, &R[size_t(r)].comm));
    });
    return R;
}

void teardown(mpixs_world w, std::vector<Rank> &R) {
    run_threads(int(R.size()), [&](int r) {
        CHECK(mpixs_comm_free(&R[size_t(r)].comm));
        CHECK(mpixs_stream_free(&R[size_t(r)].st));
        hipStreamDestroy(R[size_t(r)].hs);
    });
    int rc = mpixs_world_free(&w);
    if (rc) {
        std::fprintf(stderr, "world_free: %s\n", mpixs_error_string(rc));
        g_fail.store(1);
    }
}

std::mutex g_alloc_mu;
std::vector<void *> g_allocs;

// "device" memory of the stand-in (freed after each case)
char *dev_alloc(size_t n) {
    void *p = nullptr;
    hipMalloc(&p, n);
    std::lock_guard<std::mutex> g(g_alloc_mu);
    g_allocs.push_back(p);
    return static_cast<char *>(p);
}

void dev_free_all() {
    std::lock_guard<std::mutex> g(g_alloc_mu);
    for (void *p : g_allocs) hipFree(p);
    g_allocs.clear();
}

// ------------------------------------------------------------ patterns
void plain_batch(int reps) {
    const int n = 32, per = 40;
    mpixs_world w;
    mpixs_config cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    if (mpixs_world_create(n, &cfg, &w)) {
        g_fail.store(1);
        return;
    }
    auto R = setup(w, n);
    // message i of rank r goes to (r + 1 + i) % n with tag i % 64, and comes
    // from (r - 1 - i) mod n
    std::vector<char *> sb(static_cast<size_t>(n)), rb(static_cast<size_t>(n));
    for (int r = 0; r < n; ++r) {
        sb[size_t(r)] = dev_alloc(size_t(per) * 4096);
        rb[size_t(r)] = dev_alloc(size_t(per) * 4096);
    }
    run_threads(n, [&](int r) {
        mpixs_datatype vt;
        CHECK(mpixs_type_vector(64, 1 + r % 4, 2 * (1 + r % 4), MPIXS_FLOAT32, &vt));
        CHECK(mpixs_type_commit(&vt));
        mpixs_status *sts = reinterpret_cast<mpixs_status *>(
            dev_alloc(sizeof(mpixs_status) * size_t(2 * per)));
        for (int rep = 0; rep < reps; ++rep) {
            std::vector<mpixs_request> rq;
            for (int i = 0; i < per; ++i) {
                const int d = (r + 1 + i % (n - 1)) % n;
                mpixs_request q;
                CHECK(mpixs_isend_enqueue(sb[size_t(r)] + size_t(i) * 4096, 1000, MPIXS_UINT8, d,
                                          i % 64, R[size_t(r)].comm, &q));
                rq.push_back(q);
            }
            for (int i = 0; i < per; ++i) {
                const int s = ((r - 1 - i % (n - 1)) % n + n) % n;
                mpixs_request q;
                CHECK(mpixs_irecv_enqueue(rb[size_t(r)] + size_t(i) * 4096, 1000, MPIXS_UINT8, s,
                                          i % 64, R[size_t(r)].comm, &q));
                rq.push_back(q);
            }
            CHECK(mpixs_waitall_enqueue(int(rq.size()), rq.data(), sts));
        }
        CHECK(mpixs_type_free(&vt));
    });
    teardown(w, R);
}

void allreduces(int reps) {
    const int n = 16;
    mpixs_world w;
    if (mpixs_world_create(n, nullptr, &w)) {
        g_fail.store(1);
        return;
    }
    auto R = setup(w, n);
    std::vector<char *> in(static_cast<size_t>(n)), out(static_cast<size_t>(n));
    for (int r = 0; r < n; ++r) {
        in[size_t(r)] = dev_alloc(1 << 16);
        out[size_t(r)] = dev_alloc(1 << 16);
    }
    run_threads(n, [&](int r) {
        for (int k = 0; k < reps; ++k) {
            const int count = (k % 3 == 0) ? 16 : (1 << 14);
            CHECK(mpixs_allreduce_enqueue(k % 5 == 0 ? MPIXS_IN_PLACE : in[size_t(r)],
                                          out[size_t(r)], count,
                                          k % 2 ? MPIXS_FLOAT32 : MPIXS_INT32, MPIXS_SUM,
                                          R[size_t(r)].comm));
        }
    });
    teardown(w, R);
}

void groups_and_batches(int reps) {
    const int n = 8;
    mpixs_world w;
    if (mpixs_world_create(n, nullptr, &w)) {
        g_fail.store(1);
        return;
    }
    auto R = setup(w, n);
    std::vector<char *> a(static_cast<size_t>(n)), h(static_cast<size_t>(n)), o(static_cast<size_t>(n));
    for (int r = 0; r < n; ++r) {
        a[size_t(r)] = dev_alloc(1 << 16);
        h[size_t(r)] = dev_alloc(1 << 16);
        o[size_t(r)] = dev_alloc(1 << 16);
    }
    auto record = [&](int r, int tag) -> int {
        const int right = (r + 1) % n, left = (r + n - 1) % n;
        mpixs_request q[2];
        int rc = mpixs_group_start(R[size_t(r)].comm);
        if (!rc) rc = mpixs_isend_enqueue(a[size_t(r)], 4096, MPIXS_UINT8, right, tag, R[size_t(r)].comm, &q[0]);
        if (!rc) rc = mpixs_isend_enqueue(a[size_t(r)] + 4096, 4096, MPIXS_UINT8, left, tag, R[size_t(r)].comm, &q[1]);
        if (!rc) rc = mpixs_recv_enqueue(h[size_t(r)], 4096, MPIXS_UINT8, left, tag, R[size_t(r)].comm, nullptr);
        if (!rc) rc = mpixs_recv_enqueue(h[size_t(r)] + 4096, 4096, MPIXS_UINT8, right, tag, R[size_t(r)].comm, nullptr);
        if (!rc) rc = mpixs_waitall_enqueue(2, q, nullptr);
        if (!rc) rc = mpixs_allreduce_enqueue(a[size_t(r)] + 8192, o[size_t(r)], 512, MPIXS_FLOAT32, MPIXS_SUM, R[size_t(r)].comm);
        return rc;
    };
    run_threads(n, [&](int r) {
        for (int k = 0; k < reps; ++k) {
            CHECK(record(r, k % 64));
            CHECK(mpixs_group_end(R[size_t(r)].comm));
        }
        mpixs_batch b, bs;
        CHECK(record(r, 100));
        CHECK(mpixs_group_end_init(R[size_t(r)].comm, &b));
        for (int k = 0; k < reps; ++k) CHECK(mpixs_batch_start_enqueue(b));
        CHECK(record(r, 101));
        CHECK(mpixs_group_end_init_static(R[size_t(r)].comm, &bs));
        for (int k = 0; k < reps; ++k) CHECK(mpixs_batch_start_enqueue(bs));
        CHECK(mpixs_batch_free(&b));
        CHECK(mpixs_batch_free(&bs));
    });
    teardown(w, R);
}

void wildcards(int reps) {
    // rank 0 receives from every other rank with ANY_SOURCE / ANY_TAG (racing
// blocking senders, tags varying per iteration)
    const int n = 8;
    mpixs_world w;
    mpixs_config cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    cfg.matching = 1;
    cfg.max_channels = 256;
    if (mpixs_world_create(n, &cfg, &w)) {
        g_fail.store(1);
        return;
    }
    auto R = setup(w, n);
    char *buf = dev_alloc(1 << 20);
    run_threads(n, [&](int r) {
        mpixs_status *st = nullptr;
        if (r == 0) st = reinterpret_cast<mpixs_status *>(dev_alloc(sizeof(mpixs_status) * 64));
        for (int k = 0; k < reps; ++k) {
            if (r == 0) {
                std::vector<mpixs_request> rq(static_cast<size_t>(n - 1));
                // any receive accepts any message, so none can starve
                for (int i = 0; i < n - 1; ++i)
                    CHECK(mpixs_irecv_enqueue(buf + 8 * i, 8, MPIXS_UINT8, MPIXS_ANY_SOURCE,
                                              MPIXS_ANY_TAG, R[0].comm, &rq[size_t(i)]));
                CHECK(mpixs_waitall_enqueue(n - 1, rq.data(), st));
            } else {
                CHECK(mpixs_send_enqueue(buf + 4096 + 8 * r, 8, MPIXS_UINT8, 0, k % 5, R[size_t(r)].comm));
            }
        }
    });
    teardown(w, R);
}

void host_synced(int reps) {
    const int n = 4;
    mpixs_world w;
    if (mpixs_world_create(n, nullptr, &w)) {
        g_fail.store(1);
        return;
    }
    auto R = setup(w, n);
    char *buf = dev_alloc(1 << 20);
    run_threads(n, [&](int r) {
        for (int k = 0; k < reps; ++k) {
            if (r % 2 == 0)
                CHECK(mpixs_send(buf + 1024 * r, 256, MPIXS_UINT8, r + 1, k, R[size_t(r)].comm));
            else
                CHECK(mpixs_recv(buf + 1024 * r, 256, MPIXS_UINT8, r - 1, k, R[size_t(r)].comm, nullptr));
            CHECK(mpixs_allreduce(buf + 65536 + 1024 * r, buf + 131072 + 1024 * r, 64, MPIXS_INT64,
                                  MPIXS_MAX, R[size_t(r)].comm));
        }
    });
    teardown(w, R);
}

void create_free_cycles(int cycles) {
    const int n = 2;
    mpixs_world w;
    mpixs_config cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    cfg.max_streams = 4;
    cfg.max_collectives = 64;
    cfg.max_channels = 64;
    if (mpixs_world_create(n, &cfg, &w)) {
        g_fail.store(1);
        return;
    }
    char *buf = dev_alloc(1 << 16);
    std::atomic<int> phase{0};
    run_threads(n, [&](int r) {
        hipStream_t hs;
        hipStreamCreateWithFlags(&hs, hipStreamNonBlocking);
        mpixs_comm wc;
        CHECK(mpixs_world_comm(w, r, &wc));
        for (int c = 0; c < cycles; ++c) {
            mpixs_info info;
            mpixs_stream st;
            mpixs_comm comm;
            CHECK(mpixs_info_create(&info));
            CHECK(mpixs_info_set(info, "type", "hipStream_t"));
            CHECK(mpixs_info_set_hex(info, "value", &hs, sizeof(hs)));
            CHECK(mpixs_stream_create(w, info, &st));
            CHECK(mpixs_info_free(&info));
            CHECK(mpixs_comm_create_with_stream(wc, st, &comm));
            if (r == 0) CHECK(mpixs_send_enqueue(buf, 64, MPIXS_UINT8, 1, c, comm));
            else CHECK(mpixs_recv_enqueue(buf + 128, 64, MPIXS_UINT8, 0, c, comm, nullptr));
            CHECK(mpixs_allreduce_enqueue(buf + 256 + 64 * r, buf + 512 + 64 * r, 8, MPIXS_INT64,
                                          MPIXS_SUM, comm));
            CHECK(mpixs_comm_free(&comm));
            CHECK(mpixs_stream_free(&st));
            // both ranks finish the cycle before the next one starts
            phase.fetch_add(1);
            while (phase.load() < 2 * (c + 1)) std::this_thread::yield();
        }
        hipStreamDestroy(hs);
    });
    mpixs_stats s;
    if (!mpixs_world_get_stats(w, &s) &&
        (s.streams_recycled == 0 || s.comm_lines_recycled == 0 || s.channels_recycled == 0)) {
        std::fprintf(stderr, "cycles: nothing was recycled\n");
        g_fail.store(1);
    }
    if (mpixs_world_free(&w)) g_fail.store(1);
}

// Groups large enough that the waiting ranks help plan them: 8 ranks, each
// sending 400 messages (64 bytes, a vector type on every third) to random
// peers and receiving its own, as one-shot groups and one persistent batch.
void large_groups(int reps) {
    const int n = 8, per = 400;
    mpixs_world w;
    if (mpixs_world_create(n, nullptr, &w)) {
        g_fail.store(1);
        return;
    }
    auto R = setup(w, n);
    mpixs_datatype vt;
    CHECK(mpixs_type_vector(4, 2, 4, MPIXS_INT32, &vt));
    CHECK(mpixs_type_commit(&vt));
    // message i: from i % n to dest[i], tag i / n % 64
    std::vector<int> dest(size_t(n) * per);
    std::mt19937 g{7};
    for (size_t i = 0; i < dest.size(); ++i) dest[i] = int((i % n + 1 + g() % (n - 1)) % n);
    std::vector<char *> sb(static_cast<size_t>(n)), rb(static_cast<size_t>(n));
    for (int r = 0; r < n; ++r) {
        sb[size_t(r)] = dev_alloc(size_t(per) * 64);
        rb[size_t(r)] = dev_alloc(dest.size() * 64);
    }
    auto record = [&](int r) -> int {
        std::vector<mpixs_request> q;
        int rc = mpixs_group_start(R[size_t(r)].comm);
        for (size_t i = 0; !rc && i < dest.size(); ++i) {
            const int src = int(i % n), tag = int(i / n % 64);
            const bool vec = i % 3 == 0;
            mpixs_request x = nullptr;
            if (src == r)
                rc = mpixs_isend_enqueue(sb[size_t(r)] + (i / n) * 64, vec ? 1 : 16, vec ? vt : MPIXS_INT32,
                                         dest[i], tag, R[size_t(r)].comm, &x);
            else if (dest[i] == r)
                rc = mpixs_irecv_enqueue(rb[size_t(r)] + i * 64, vec ? 1 : 16, vec ? vt : MPIXS_INT32,
                                         src, tag, R[size_t(r)].comm, &x);
            if (x) q.push_back(x);
        }
        if (!rc) rc = mpixs_waitall_enqueue(int(q.size()), q.data(), nullptr);
        return rc;
    };
    run_threads(n, [&](int r) {
        for (int k = 0; k < reps; ++k) {
            CHECK(record(r));
            CHECK(mpixs_group_end(R[size_t(r)].comm));
        }
        mpixs_batch b;
        CHECK(record(r));
        CHECK(mpixs_group_end_init(R[size_t(r)].comm, &b));
        for (int k = 0; k < reps; ++k) CHECK(mpixs_batch_start_enqueue(b));
        CHECK(mpixs_batch_free(&b));
    });
    CHECK(mpixs_type_free(&vt));
    teardown(w, R);
}

void types_everywhere(int reps) {
    run_threads(8, [&](int t) {
        std::mt19937 g{static_cast<uint32_t>(t)};
        for (int k = 0; k < reps; ++k) {
            mpixs_datatype a, b;
            CHECK(mpixs_type_vector(1 + int(g() % 50), 1 + int(g() % 4), 8, MPIXS_INT32, &a));
            int bls[3] = {1, 2, 3}, ds[3] = {0, 4, 9};
            CHECK(mpixs_type_indexed(3, bls, ds, a, &b));
            CHECK(mpixs_type_commit(&b));
            int64_t sz, lb, ext;
            CHECK(mpixs_type_size(b, &sz));
            CHECK(mpixs_type_get_extent(b, &lb, &ext));
            CHECK(mpixs_type_free(&b));
            CHECK(mpixs_type_free(&a));
        }
    });
}

}  // namespace

int main(int argc, char **argv) {
    const int scale = argc > 1 ? std::atoi(argv[1]) : 1;
    struct {
        const char *name;
        std::function<void()> f;
    } cases[] = {
        {"plain batch, 32 ranks", [&] { plain_batch(3 * scale); }},
        {"enqueued allreduces, 16 ranks", [&] { allreduces(60 * scale); }},
        {"groups and persistent batches, 8 ranks", [&] { groups_and_batches(20 * scale); }},
        {"large groups planned with help, 8 ranks", [&] { large_groups(4 * scale); }},
        {"wildcard receives, 8 ranks", [&] { wildcards(30 * scale); }},
        {"host-synchronised calls, 4 ranks", [&] { host_synced(30 * scale); }},
        {"stream and communicator cycles", [&] { create_free_cycles(300 * scale); }},
        {"datatypes from 8 threads", [&] { types_everywhere(200 * scale); }},
    };
    for (auto &c : cases) {
        std::printf("[case] %s\n", c.name);
        std::fflush(stdout);
        c.f();
        dev_free_all();
        if (g_fail.load()) {
            std::printf("FAILED in %s\n", c.name);
            return 1;
        }
    }
    std::printf("ok (%llu launches recorded)\n", (unsigned long long)hipstub_launches());
    return 0;
}
