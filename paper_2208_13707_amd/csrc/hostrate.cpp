// Host analog of the paper's multithreaded message-rate measurement (§5.3,
// Fig. 3).  Two simulated processes, a sender side A and a receiver side B,
// each hold one communication context (VCI) per thread; thread i of A sends
// 8-byte messages to thread i of B with isend / irecv in windows closed by a
// waitall.  The wire between context A_i and B_i is a single-producer /
// single-consumer ring (it stands for the network, and is lock-free in every
// mode).  The message engine above the wire -- request objects, the posted
// and unexpected queues, the progress loop -- is synchronised by one of
// three policies:
//
//   0  global critical section: one mutex per process, held for the whole of
//      every call, released and retaken only between progress-loop passes of
//      a waitall (§2.1);
//   1  per-context critical sections: one mutex per context, taken
//      separately on the send path, the receive path, every progress pass
//      and every request release (§2.2, §5.3), so a message crosses several
//      critical sections even when no other thread contends for them;
//   2  stream contexts: a stream is a strictly serial execution context, so
//      the engine takes no lock at all (§3.1).
//
// Request reference counts and completion flags stay atomic in every mode,
// as in the paper's implementation (§5.3).  This is a CPU-only model of the
// engine's synchronisation cost; it does not touch the GPU.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/mpixs_driver.h"

namespace {

constexpr int kMaxWindow = 1024;
constexpr int kRing = 2 * kMaxWindow;   // two windows may be in flight

inline void cpu_relax() { __builtin_ia32_pause(); }

struct Request {
    std::atomic<int> refs{0};
    std::atomic<int> complete{0};
    uint64_t *dst = nullptr;   // receive buffer (receive requests)
};

struct alignas(64) WireSlot {
    std::atomic<uint32_t> full{0};
    uint64_t payload = 0;
};

struct Wire {   // A_i -> B_i
    WireSlot slot[kRing];
    alignas(64) uint64_t head = 0;   // producer position (side A only)
    alignas(64) uint64_t tail = 0;   // consumer position (side B only)
};

struct alignas(64) Context {
    std::mutex mu;                        // policy 1
    std::vector<Request *> pool;          // free request objects
    std::vector<std::unique_ptr<Request>> owned;
    std::deque<Request *> posted;         // receive side: posted receives
    std::deque<uint64_t> unexpected;      // receive side: arrived, unmatched
    Wire *wire = nullptr;

    Context() {
        for (int k = 0; k < 2 * kMaxWindow; ++k) {
            owned.emplace_back(new Request());
            pool.push_back(owned.back().get());
        }
    }
};

struct Process {
    alignas(64) std::mutex global;   // policy 0 (own cache line: no false sharing)
    alignas(64) std::vector<std::unique_ptr<Context>> ctx;
};

struct alignas(64) Ack {   // windows received on one pair
    std::atomic<int64_t> n{0};
};

// A critical section of the given policy: the global mutex (policy 0, only
// where the caller asks for it), the context's mutex (policy 1), or none.
class Section {
public:
    Section(int policy, Process &p, Context &c, bool global_here)
        : m_(policy == 1 ? &c.mu : (policy == 0 && global_here ? &p.global : nullptr)) {
        if (m_) m_->lock();
    }
    ~Section() {
        if (m_) m_->unlock();
    }
    Section(const Section &) = delete;
    Section &operator=(const Section &) = delete;

private:
    std::mutex *m_;
};

// Request allocation: one reference for the user, one for the engine.
Request *alloc_request(Context &c) {
    Request *r = c.pool.back();
    c.pool.pop_back();
    r->complete.store(0, std::memory_order_relaxed);
    r->refs.store(2, std::memory_order_relaxed);
    return r;
}

void release_ref(Context &c, Request *r) {
    if (r->refs.fetch_sub(1, std::memory_order_acq_rel) == 1) c.pool.push_back(r);
}

// Progress on a receive context: drain the wire, matching arrivals against
// posted receives in order (non-overtaking), else queueing them as unexpected.
void progress_recv(Context &c) {
    Wire &w = *c.wire;
    for (;;) {
        WireSlot &s = w.slot[w.tail % kRing];
        if (!s.full.load(std::memory_order_acquire)) break;
        const uint64_t v = s.payload;
        s.full.store(0, std::memory_order_release);
        ++w.tail;
        if (!c.posted.empty()) {
            Request *r = c.posted.front();
            c.posted.pop_front();
            *r->dst = v;
            r->complete.store(1, std::memory_order_release);
            release_ref(c, r);
        } else {
            c.unexpected.push_back(v);
        }
    }
}

struct Bench {
    int policy;
    int window;
    int64_t per_pair;
    Process a, b;
    std::vector<std::unique_ptr<Wire>> wires;
    std::vector<std::unique_ptr<Ack>> acked;

    // The sender's isend: eager injection into the wire, completing at once.
    // Returns nullptr while the wire is full (never inside a window, since the
    // sender waits for the window before last to be received).
    Request *isend(Context &c, uint64_t v) {
        Section cs(policy, a, c, true);
        Wire &w = *c.wire;
        WireSlot &s = w.slot[w.head % kRing];
        if (s.full.load(std::memory_order_acquire)) return nullptr;
        Request *r = alloc_request(c);
        s.payload = v;
        s.full.store(1, std::memory_order_release);
        ++w.head;
        r->complete.store(1, std::memory_order_release);
        release_ref(c, r);
        return r;
    }

    Request *irecv(Context &c, uint64_t *dst) {
        Section cs(policy, b, c, true);
        Request *r = alloc_request(c);
        r->dst = dst;
        if (!c.unexpected.empty()) {
            *dst = c.unexpected.front();
            c.unexpected.pop_front();
            r->complete.store(1, std::memory_order_release);
            release_ref(c, r);
        } else {
            c.posted.push_back(r);
        }
        return r;
    }

    // waitall over n requests of one context of process p.
    void waitall(Process &p, Context &c, Request **reqs, int n, bool recv_side) {
        if (policy == 0) {
            // one critical section for the call, yielded between passes
            std::unique_lock<std::mutex> g(p.global);
            for (;;) {
                if (recv_side) progress_recv(c);
                bool all = true;
                for (int k = 0; k < n && all; ++k)
                    all = reqs[k]->complete.load(std::memory_order_acquire) != 0;
                if (all) break;
                g.unlock();
                cpu_relax();
                g.lock();
            }
            for (int k = 0; k < n; ++k) release_ref(c, reqs[k]);
            return;
        }
        for (int k = 0; k < n; ++k) {
            while (!reqs[k]->complete.load(std::memory_order_acquire)) {
                if (recv_side) {
                    Section cs(policy, p, c, false);
                    progress_recv(c);
                } else {
                    cpu_relax();
                }
            }
            Section cs(policy, p, c, false);
            release_ref(c, reqs[k]);
        }
    }

    void sender(int i) {
        Context &c = *a.ctx[size_t(i)];
        std::vector<Request *> reqs(static_cast<size_t>(window));
        int64_t n = 0, win = 0;
        while (n < per_pair) {
            // at most two windows in flight
            while (acked[size_t(i)]->n.load(std::memory_order_acquire) < win - 1) cpu_relax();
            const int w = int(std::min<int64_t>(window, per_pair - n));
            for (int k = 0; k < w; ++k) {
                Request *r;
                while (!(r = isend(c, uint64_t(i) << 40 | uint64_t(n + k)))) cpu_relax();
                reqs[size_t(k)] = r;
            }
            waitall(a, c, reqs.data(), w, false);
            n += w;
            ++win;
        }
    }

    uint64_t receiver(int i) {
        Context &c = *b.ctx[size_t(i)];
        std::vector<Request *> reqs(static_cast<size_t>(window));
        std::vector<uint64_t> buf(static_cast<size_t>(window));
        uint64_t sum = 0;
        int64_t n = 0;
        while (n < per_pair) {
            const int w = int(std::min<int64_t>(window, per_pair - n));
            for (int k = 0; k < w; ++k) reqs[size_t(k)] = irecv(c, &buf[size_t(k)]);
            waitall(b, c, reqs.data(), w, true);
            for (int k = 0; k < w; ++k) sum += buf[size_t(k)] * uint64_t(n + k + 1);
            n += w;
            acked[size_t(i)]->n.fetch_add(1, std::memory_order_release);
        }
        return sum;
    }
};

}  // namespace

extern "C" int mpixs_drv_host_msgrate(int npairs, int policy, int64_t msgs_per_pair, int window,
                                      double *msgs_per_s, uint64_t *checksum) {
    if (npairs <= 0 || npairs > 256 || policy < 0 || policy > 2 || msgs_per_pair <= 0 ||
        window <= 0 || window > kMaxWindow || !msgs_per_s)
        return 1;
    Bench e;
    e.policy = policy;
    e.window = window;
    e.per_pair = msgs_per_pair;
    for (int i = 0; i < npairs; ++i) {
        e.wires.emplace_back(new Wire());
        e.acked.emplace_back(new Ack());
        e.a.ctx.emplace_back(new Context());
        e.b.ctx.emplace_back(new Context());
        e.a.ctx.back()->wire = e.wires.back().get();
        e.b.ctx.back()->wire = e.wires.back().get();
    }
    std::atomic<int> ready{0}, go{0};
    std::vector<uint64_t> sums(size_t(npairs), 0);
    std::vector<std::thread> th;
    auto start = [&] {
        ready.fetch_add(1);
        while (!go.load(std::memory_order_acquire)) std::this_thread::yield();
    };
    for (int i = 0; i < npairs; ++i) {
        th.emplace_back([&, i] {
            start();
            e.sender(i);
        });
        th.emplace_back([&, i] {
            start();
            sums[size_t(i)] = e.receiver(i);
        });
    }
    while (ready.load() < 2 * npairs) std::this_thread::yield();
    const auto t0 = std::chrono::steady_clock::now();
    go.store(1, std::memory_order_release);
    for (auto &t : th) t.join();
    const double sec =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *msgs_per_s = double(npairs) * double(msgs_per_pair) / sec;
    if (checksum) {
        uint64_t s = 0;
        for (uint64_t x : sums) s += x;
        *checksum = s;
    }
    return 0;
}
