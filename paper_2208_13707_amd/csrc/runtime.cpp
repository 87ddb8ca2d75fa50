// libmpixs host runtime: worlds, info, streams, stream communicators and
// the enqueue protocol.
//
// Matching (§2.1).  A channel is (communicator, source, destination, tag).
// The source thread numbers its sends on a channel 0, 1, 2 ... and the
// destination thread numbers its receives the same way; send k matches
// receive k.  Because a stream is a strictly serial context used by one
// thread (§3.1), the two counters need no lock.
//
// Enqueue protocol (§3.4).  For message k the side whose thread arrives
// first enqueues a one-thread "post" kernel that stores ready[side] = k+1
// when its stream reaches the operation, then records its descriptor.  The
// side that arrives second enqueues, on its own stream, the copy: wait until
// the other side's ready counter reaches k+1, move the bytes from the
// sender's typemap into the receiver's, publish done = k+1.  The first side
// later (blocking call: at once; nonblocking call: at its wait) enqueues a
// one-wave wait for done >= k+1, after the copy has been enqueued.
//
// So every device wait is enqueued after the work it waits for.  HIP maps
// streams onto a few hardware queues that run their packets in order, so a
// wait queued ahead of its producer on a shared queue could never finish;
// with this rule the earliest unfinished packet never waits for a later one
// and the system always makes progress.  The price is that a call may wait
// on the host until the peer thread has *enqueued* its side (never until
// any GPU work has finished).
//
// Allreduce: the last rank to arrive runs the whole reduction on its
// stream after waiting for the other ranks' arrive counters; the others
// post their arrival and wait for the done counter.
#include <hip/hip_runtime.h>

#include <immintrin.h>
#include <linux/futex.h>
#include <sys/syscall.h>
#include <unistd.h>

#include <cerrno>
#include <climits>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <thread>
#include <tuple>
#include <vector>

#include "mpixs_launch.h"
#include "runtime.h"
#include "../../include/mpixs_debug.h"

namespace mpixs {

namespace {

constexpr uint64_t kModeHost = uint64_t(1) << 63;

// Largest grid of a fused kernel, whose workgroups poll before they work.
// With at most 32 hardware queues per process (one running kernel each),
// polling workgroups hold at most 32 * 32 * 4 = 4096 of the chip's 8192+
// wave slots, so the kernels they wait for always find room.
constexpr uint64_t kFusedMaxWG = 32;

int gpu_err(hipError_t e) { return e == hipSuccess ? MPIXS_SUCCESS : MPIXS_ERR_GPU; }

// Distinct (source, destination, tag) give distinct keys: ranks are below
// 4096 (12 bits each, bits 44..55 and 32..43), tags below 2^31 (bits
// 0..30); bit 63 is left for the host-synchronised mode.
uint64_t chan_key(int src, int dst, int tag) {
    return (uint64_t(uint32_t(src)) << 44) | (uint64_t(uint32_t(dst)) << 32) | uint64_t(uint32_t(tag));
}

// Host sleeping.  Rank threads often outnumber the host's cores, so a
// thread that waits for another thread's enqueue must not hold a core for
// long: it spins briefly, then yields its core for up to kYieldUs, then
// sleeps on a futex word chosen by the address of the object it waits on (a
// hashed table); whoever changes such an object bumps that word and wakes
// its sleepers -- a system call only when someone sleeps there.  The waiter reads the word before testing its predicate and
// the kernel compares it again before sleeping, so a change between the two
// is never missed; sleeps are also bounded (1 ms), and abort wakes everyone.
struct alignas(64) WakeSlot {
    std::atomic<uint32_t> seq{0};
    std::atomic<uint32_t> sleepers{0};
};
constexpr int kWakeSlots = 1024;
WakeSlot g_wake[kWakeSlots];

WakeSlot &wake_slot(const void *key) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(key);
    return g_wake[((x >> 6) ^ (x >> 16)) & (kWakeSlots - 1)];
}

void futex_wake_all(std::atomic<uint32_t> *word) {
    syscall(SYS_futex, reinterpret_cast<uint32_t *>(word), FUTEX_WAKE_PRIVATE, INT32_MAX, nullptr,
            nullptr, 0);
}

void host_notify(const void *key) {
    WakeSlot &s = wake_slot(key);
    s.seq.fetch_add(1, std::memory_order_seq_cst);
    if (s.sleepers.load(std::memory_order_seq_cst) != 0) futex_wake_all(&s.seq);
}

void host_notify_all() {
    for (WakeSlot &s : g_wake) {
        s.seq.fetch_add(1, std::memory_order_seq_cst);
        if (s.sleepers.load(std::memory_order_seq_cst) != 0) futex_wake_all(&s.seq);
    }
}

// Wait on the host until pred() holds; `key` is the address of the object
// pred() reads (its writer calls host_notify(key)).  Gives up on abort or
// after the world's timeout (which aborts the world so that every device
// wait ends too).
template <class Pred>
int host_wait(World *w, const void *key, Pred pred) {
    if (pred()) return MPIXS_SUCCESS;
    w->host_waits.fetch_add(1, std::memory_order_relaxed);
    for (int i = 0; i < 128; ++i) {
        _mm_pause();
        if (pred()) return MPIXS_SUCCESS;
    }
    const auto t0 = std::chrono::steady_clock::now();
    constexpr auto kYieldUs = std::chrono::microseconds(50);
    while (std::chrono::steady_clock::now() - t0 < kYieldUs) {
        std::this_thread::yield();
        if (pred()) return MPIXS_SUCCESS;
    }
    WakeSlot &s = wake_slot(key);
    const auto limit = std::chrono::milliseconds(w->cfg.timeout_ms);
    w->host_sleeps.fetch_add(1, std::memory_order_relaxed);
    for (;;) {
        const uint32_t seq = s.seq.load(std::memory_order_seq_cst);
        if (pred()) return MPIXS_SUCCESS;
        if (w->aborted.load(std::memory_order_acquire)) return MPIXS_ERR_ABORTED;
        if (std::chrono::steady_clock::now() - t0 > limit) {
            mpixs_world_abort(reinterpret_cast<mpixs_world>(w));
            return MPIXS_ERR_TIMEOUT;
        }
        s.sleepers.fetch_add(1, std::memory_order_seq_cst);
        struct timespec ts = {0, 1000000};
        const long r = syscall(SYS_futex, reinterpret_cast<uint32_t *>(&s.seq), FUTEX_WAIT_PRIVATE,
                               seq, &ts, nullptr, 0);
        if (r != 0 && errno == ETIMEDOUT)
            w->host_sleep_timeouts.fetch_add(1, std::memory_order_relaxed);
        s.sleepers.fetch_sub(1, std::memory_order_seq_cst);
    }
}

WaitCtl ctl_of(World *w) {
    WaitCtl c;
    c.abort = w->h_abort;
    c.timeout_ticks = w->timeout_ticks;
    return c;
}

bool profile_on(World *w) { return w->cfg.profile != 0; }

void prof_begin(World *, hipStream_t s, hipEvent_t *e0) {
    (void)hipEventCreate(e0);
    (void)hipEventRecord(*e0, s);
}

void prof_end(World *w, hipStream_t s, hipEvent_t e0, int kind) {
    hipEvent_t e1;
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e1, s);
    std::lock_guard<std::mutex> g(w->prof_mu);
    w->prof.push_back(ProfPair{e0, e1, kind});
}

// ------------------------------------------------------------------ maps
int64_t lowbit(int64_t g) { return g ? (g & -g) : int64_t(1) << 62; }

// One side of a copy: the map kind and base, and `g`, the OR of every
// quantity the unit size must divide (its lowest set bit bounds the unit).
struct MapPlan {
    DMap m{};
    int64_t g = 0;
};

void plan_map(const Side &sd, MapPlan &p) {
    const Layout &L = sd.t->L;
    const uint64_t buf = reinterpret_cast<uint64_t>(sd.buf);
    std::memset(&p.m, 0, sizeof(p.m));
    if (L.reg && L.nblk == 1) {
        // count copies of a dense block are one dense run
        p.m.kind = MAP_CONTIG;
        p.m.base = buf + uint64_t(L.first);
        p.g = int64_t(p.m.base);
        return;
    }
    if (L.reg) {
        p.m.kind = MAP_VEC;
        p.m.base = buf + uint64_t(L.first);
        p.m.s_blk = L.stride;
        p.m.s_copy = L.extent;
        int64_t g = int64_t(p.m.base) | L.blen | (L.stride < 0 ? -L.stride : L.stride);
        if (sd.count > 1) g |= L.extent;
        p.g = g;
        return;
    }
    p.m.kind = MAP_SEG;
    p.m.base = buf;
    p.m.s_copy = L.extent;
    p.m.seg = sd.t->table;
    p.m.nseg = uint32_t(sd.t->nseg);
    p.m.lut = sd.t->lut;
    p.m.bu = sd.t->lut_shift;
    int64_t g = int64_t(buf) | L.gcd;
    if (sd.count > 1) g |= L.extent;
    p.g = g;
}

void finish_map(const Side &sd, MapPlan &p, int w, uint64_t units) {
    const Layout &L = sd.t->L;
    if (p.m.kind == MAP_VEC) {
        p.m.bu = uint32_t(L.blen / w);
        const bool periodic = sd.count == 1 || L.extent == L.nblk * L.stride;
        p.m.upc = periodic ? uint32_t(std::max<uint64_t>(units, 1)) : uint32_t(L.nblk * (L.blen / w));
        if (periodic) p.m.s_copy = 0;
        p.m.d_bu = make_fastdiv(std::max<uint32_t>(p.m.bu, 1));
        p.m.d_upc = make_fastdiv(std::max<uint32_t>(p.m.upc, 1));
    } else if (p.m.kind == MAP_SEG) {
        p.m.upc = uint32_t(L.size / w);
        p.m.d_upc = make_fastdiv(std::max<uint32_t>(p.m.upc, 1));
    }
}

}  // namespace

int plan_copy(const Side &S, const Side &R, int64_t nbytes, DMap *src, DMap *dst, int *wsz,
              uint64_t *units, uint32_t *tail) {
    MapPlan ps, pr;
    *wsz = 16;
    *units = 0;
    if (tail) *tail = 0;
    if (nbytes <= 0) {
        std::memset(src, 0, sizeof(*src));
        std::memset(dst, 0, sizeof(*dst));
        return MPIXS_SUCCESS;
    }
    plan_map(S, ps);
    plan_map(R, pr);
    if (tail && ps.m.kind == MAP_CONTIG && pr.m.kind == MAP_CONTIG) {
        // dense on both sides: the unit follows the base addresses alone and
        // the last nbytes mod W bytes form a byte tail
        *wsz = int(std::min<int64_t>(16, lowbit(ps.g | pr.g)));
        *units = uint64_t(nbytes / *wsz);
        *tail = uint32_t(nbytes % *wsz);
        finish_map(S, ps, *wsz, *units);
        finish_map(R, pr, *wsz, *units);
        *src = ps.m;
        *dst = pr.m;
        return MPIXS_SUCCESS;
    }
    const int64_t g = nbytes | ps.g | pr.g;
    *wsz = int(std::min<int64_t>(16, lowbit(g)));
    *units = uint64_t(nbytes / *wsz);
    finish_map(S, ps, *wsz, *units);
    finish_map(R, pr, *wsz, *units);
    *src = ps.m;
    *dst = pr.m;
    return MPIXS_SUCCESS;
}

namespace {

StatusVal match_status(const Side &s, const Side &r, int tag) {
    StatusVal st{};
    st.source = s.rank;
    st.tag = tag;
    st.source_index = s.idx;   // the sender's stream index (multiplex communicators)
    const int64_t cap = r.bytes;
    if (s.bytes > 0 && cap > 0 && s.t->L.basic != r.t->L.basic) {
        st.error = MPIXS_ERR_TYPE;
        st.count_bytes = 0;
    } else if (s.bytes > cap) {
        st.error = MPIXS_ERR_TRUNCATE;
        st.count_bytes = cap;
    } else {
        st.error = MPIXS_SUCCESS;
        st.count_bytes = s.bytes;
    }
    return st;
}

// ------------------------------------------------------------- launchers
// The stream block a kernel records trace events through, or nullptr when
// the world does not trace; and a trace kind, or 0 when it does not.
DevStream *trace_of(const World *w, const StreamObj *st) { return w->d_trace ? st->dev : nullptr; }
uint32_t trace_kind(const World *w, uint32_t kind) { return w->d_trace ? kind : 0; }

int do_post(World *w, StreamObj *st, uint64_t *p, uint64_t v) {
    w->n_post.fetch_add(1, std::memory_order_relaxed);
    return gpu_err(launch_post(st->hs, p, v, trace_of(w, st)));
}

// kind: what a passing lane records (MPIXS_TRACE_MATCH for a wait on a
// peer's post, MPIXS_TRACE_COMPLETE for a wait on a completion)
int do_wait(World *w, StreamObj *st, WaitArgs &a, uint32_t kind) {
    a.ctl = ctl_of(w);
    a.me = st->dev;
    a.trace = trace_kind(w, kind);
    w->n_wait.fetch_add(1, std::memory_order_relaxed);
    return gpu_err(launch_wait(st->hs, a));
}

WaitArgs wait_one(const uint64_t *p, uint64_t target) {
    WaitArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = 1;
    a.ptr[0] = p;
    a.target[0] = target;
    return a;
}

// What a copy's completion writes besides done: a host flag set to 1 once
// nothing reads the source any more (eager staging), and a channel block's
// release word (the copy is the block's last device use).
struct CopyExtra {
    uint32_t *host_flag = nullptr;
    uint64_t *rel_word = nullptr;
    uint64_t rel_val = 0;
};

// Copy message S -> R on stream `on`.  wait_ptr/target: the other side's
// ready counter (nullptr on the host-synchronised path).  done_ptr: the
// channel's done counter (nullptr: none).  status/set_error: the receive
// status and sticky error when `on` is the receiver's stream.
int do_copy(World *w, StreamObj *on, const Side &S, const Side &R, const StatusVal &st,
            const uint64_t *wait_ptr, uint64_t wait_target, uint64_t *done_ptr, uint64_t done_val,
            void *status, bool set_error, const CopyExtra *x = nullptr) {
    const int64_t nbytes = st.count_bytes;
    DMap ms, mr;
    int wsz = 16;
    uint64_t units = 0;
    plan_copy(S, R, nbytes, &ms, &mr, &wsz, &units);
    const bool fuse = w->cfg.fuse_max_bytes >= 0 && nbytes <= w->cfg.fuse_max_bytes;
    const uint64_t per_chunk = uint64_t(copy_block_units(fuse));
    const uint64_t nchunks = std::max<uint64_t>(1, (units + per_chunk - 1) / per_chunk);
    CopyArgs a;
    std::memset(&a, 0, sizeof(a));
    a.src = ms;
    a.dst = mr;
    a.units = units;
    a.ctl = ctl_of(w);
    a.me = on->dev;
    int rc = MPIXS_SUCCESS;
    hipEvent_t e0 = nullptr;
    if (fuse) {
        // one kernel: wait, copy, publish (bounded grid, see kFusedMaxWG)
        const uint64_t nwg = std::min<uint64_t>(nchunks, kFusedMaxWG);
        a.wait_ptr = wait_ptr;
        a.wait_target = wait_target;
        a.done_ptr = done_ptr;
        a.done_val = done_val;
        a.ticket_last = on->tickets + nwg - 1;
        a.status = status;
        a.st = st;
        a.set_error = set_error ? 1 : 0;
        a.trace = trace_kind(w, 1);
        if (x) {
            a.host_flag = x->host_flag;
            a.rel_word = x->rel_word;
            a.rel_val = x->rel_val;
        }
        if (profile_on(w)) prof_begin(w, on->hs, &e0);
        rc = gpu_err(launch_copy(on->hs, a, wsz, int(nwg), true));
        if (profile_on(w)) prof_end(w, on->hs, e0, 0);
        if (rc) return rc;
        if (nwg > 1) on->tickets += nwg;
    } else {
        // wait kernel, full-grid data kernel, signal kernel
        if (wait_ptr) {
            WaitArgs wa = wait_one(wait_ptr, wait_target);
            rc = do_wait(w, on, wa, MPIXS_TRACE_MATCH);
            if (rc) return rc;
        }
        if (units > 0) {
            const uint64_t nwg = std::min<uint64_t>(nchunks, uint64_t(1) << 22);
            if (profile_on(w)) prof_begin(w, on->hs, &e0);
            rc = gpu_err(launch_copy(on->hs, a, wsz, int(nwg), false));
            if (profile_on(w)) prof_end(w, on->hs, e0, 0);
            if (rc) return rc;
        }
        if (done_ptr || status || (set_error && st.error) || x) {
            SignalArgs sg;
            std::memset(&sg, 0, sizeof(sg));
            sg.done_ptr = done_ptr;
            sg.done_val = done_val;
            sg.me = on->dev;
            sg.status = status;
            sg.st = st;
            sg.set_error = set_error ? 1 : 0;
            sg.trace = trace_kind(w, 1);
            if (x) {
                sg.host_flag = x->host_flag;
                sg.rel_word = x->rel_word;
                sg.rel_val = x->rel_val;
            }
            rc = gpu_err(launch_signal(on->hs, sg));
            if (rc) return rc;
            w->n_post.fetch_add(1, std::memory_order_relaxed);
        }
    }
    w->n_copy.fetch_add(1, std::memory_order_relaxed);
    w->bytes_copied.fetch_add(uint64_t(nbytes), std::memory_order_relaxed);
    return MPIXS_SUCCESS;
}

// Reserve `bytes` of the eager staging ring and a completion flag, or give
// up at once when the ring is full: the send then takes the rendezvous
// protocol, so no sender ever waits for staging.  Slots are recycled in
// order once the receiver's copy has set their flags.
bool stage_alloc(World *w, size_t bytes, uint8_t **ptr, int *flag) {
    World::StageRing &g = w->stage;
    if (!g.base) return false;
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes > g.bytes) return false;
    std::lock_guard<std::mutex> lk(g.mu);
    while (!g.live.empty() && __atomic_load_n(&g.flags[g.live.front().flag], __ATOMIC_ACQUIRE) == 1) {
        g.free_flags.push_back(g.live.front().flag);
        g.live.pop_front();
    }
    if (g.live.empty()) g.head = 0;
    if (g.free_flags.empty()) return false;
    size_t at = 0;
    if (!g.live.empty()) {
        const size_t tail = g.live.front().off;
        if (g.head >= tail) {
            if (g.head + bytes <= g.bytes) at = g.head;
            else if (bytes < tail) at = 0;
            else return false;
        } else if (g.head + bytes < tail) {
            at = g.head;
        } else {
            return false;
        }
    }
    const int f = g.free_flags.back();
    g.free_flags.pop_back();
    __atomic_store_n(&g.flags[f], 0u, __ATOMIC_RELEASE);
    g.live.push_back(World::ArenaUse{at, bytes, f});
    g.head = at + bytes;
    *ptr = g.base + at;
    *flag = f;
    return true;
}

// A staging slot that no kernel will read (its launch failed) is free again.
void stage_drop(World *w, int flag) {
    __atomic_store_n(&w->stage.flags[flag], 1u, __ATOMIC_RELEASE);
}

// The packed bytes of an eager send in staging, as a contiguous side.
Side stage_side(uint8_t *stage, int64_t bytes, int rank) {
    Side p;
    p.buf = stage;
    p.count = int(bytes);
    p.t = type_lookup(MPIXS_UINT8);
    p.bytes = bytes;
    p.rank = rank;
    return p;
}

// --------------------------------------------------------------- channels
Channel *get_channel(mpixs_comm_s *c, int src, int dst, int tag, bool host_mode) {
    const uint64_t key = chan_key(src, dst, tag) | (host_mode ? kModeHost : 0);
    auto it = c->cache.find(key);
    if (it != c->cache.end()) return it->second;
    CommShared *sh = c->sh;
    Channel *ch = nullptr;
    {
        std::lock_guard<std::mutex> g(sh->dir_mu);
        auto jt = sh->dir.find(key);
        if (jt != sh->dir.end()) {
            ch = jt->second;
        } else {
            // the device block is attached by the first enqueued message
            ch = new Channel();
            ch->owner = sh;
            sh->dir.emplace(key, ch);
        }
    }
    c->cache.emplace(key, ch);
    return ch;
}

void rec_release(Channel *ch, Rec *r) {
    if (r->refs.fetch_sub(1, std::memory_order_acq_rel) == 1) {
        if (ch->priv) {
            delete ch;   // a one-message channel dies with its message
            return;
        }
        std::lock_guard<std::mutex> g(ch->mu);
        ch->collect();
    }
}

// ------------------------------------------------------- block recycling
// Move blocks whose last device user has written their release word to the
// free list.  Caller holds w->chan_mu.  A block still attached to a channel
// is detached only if the channel's lock is free at once (the caller may
// hold another channel's lock) and nothing was issued on the channel since
// it became quiescent.
void reclaim_blocks(World *w) {
    auto released = [&](uint32_t idx, uint64_t v) {
        return __atomic_load_n(&w->h_rel[idx], __ATOMIC_ACQUIRE) == v;
    };
    size_t j = 0;
    for (size_t i = 0; i < w->chan_limbo.size(); ++i) {
        const auto e = w->chan_limbo[i];
        if (released(e.first, e.second)) w->chan_free.push_back(e);
        else w->chan_limbo[j++] = e;
    }
    w->chan_limbo.resize(j);
    j = 0;
    for (size_t i = 0; i < w->chan_drain.size(); ++i) {
        Channel *ch = w->chan_drain[i];
        bool keep = true;
        if (ch->mu.try_lock()) {
            if (ch->idx == kNoBlock || ch->seq[0] != ch->drain_seq || ch->seq[1] != ch->drain_seq) {
                keep = false;   // issued on since: a later wait marks it again
            } else if (released(ch->idx, ch->drain_val)) {
                w->chan_free.emplace_back(ch->idx, ch->drain_val);
                ch->idx = kNoBlock;
                ch->d = nullptr;
                keep = false;
            }
            if (!keep) ch->draining = false;
            ch->mu.unlock();
        }
        if (keep) w->chan_drain[j++] = ch;
    }
    w->chan_drain.resize(j);
}

// Attach a device block to a channel whose next message is number k.
// Caller holds ch->mu (or owns a channel nobody else sees yet).  Takes a
// recycled block first, then a fresh one; with the pool exhausted it waits
// up to the world's timeout for blocks whose releases are already enqueued
// or held by eager messages whose receives are still to come.
// MPIXS_ERR_NOMEM when none can come.
int attach_block(World *w, Channel *ch, uint64_t k) {
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        {
            std::lock_guard<std::mutex> g(w->chan_mu);
            uint32_t idx = kNoBlock;
            uint64_t floor = 0;
            if (w->chan_free.empty() && w->chan_next.load(std::memory_order_relaxed) >= w->chan_cap)
                reclaim_blocks(w);
            if (!w->chan_free.empty()) {
                idx = w->chan_free.back().first;
                floor = w->chan_free.back().second;
                w->chan_free.pop_back();
                w->chans_recycled.fetch_add(1, std::memory_order_relaxed);
            } else if (w->chan_next.load(std::memory_order_relaxed) < w->chan_cap) {
                idx = w->chan_next.fetch_add(1);
            }
            if (idx != kNoBlock) {
                ch->idx = idx;
                ch->d = w->d_chans + idx;
                ch->ebase = floor;
                ch->kbase = k;
                return MPIXS_SUCCESS;
            }
            // blocks can still come from releases already enqueued, or from
            // eager messages once their receives are enqueued
            if (w->chan_limbo.empty() && w->chan_drain.empty() &&
                w->eager_held.load(std::memory_order_relaxed) == 0)
                return MPIXS_ERR_NOMEM;
        }
        if (w->aborted.load()) return MPIXS_ERR_ABORTED;
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(w->cfg.timeout_ms))
            return MPIXS_ERR_NOMEM;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

// The first side's wait for message k is the message's last device use.
// It may release the block when the channel is one message's, or when
// nothing else has been issued on the channel (quiescent after k).
bool want_release(Channel *ch, const Rec *rec, uint64_t k) {
    if (ch->priv) return true;
    std::lock_guard<std::mutex> g(ch->mu);
    return ch->seq[0] == k + 1 && ch->seq[1] == k + 1 && ch->idx == rec->didx;
}

// After the releasing wait is enqueued: record what its release word will
// read once it has passed.
void note_release(World *w, Channel *ch, const Rec *rec, uint64_t k) {
    std::lock_guard<std::mutex> g(w->chan_mu);
    if (ch->priv) {
        w->chan_limbo.emplace_back(rec->didx, rec->dv);
        return;
    }
    if (k + 1 < ch->drain_seq) return;
    ch->drain_seq = k + 1;
    ch->drain_val = rec->dv;
    if (!ch->draining) {
        ch->draining = true;
        w->chan_drain.push_back(ch);
    }
}

void set_rec_block(Channel *ch, Rec *rec, uint64_t k) {
    if (!rec->d) {
        rec->d = ch->d;
        rec->didx = ch->idx;
        rec->dv = ch->dval(k);
    }
}

bool type_ok(mpixs_datatype dt, const TypeObj **t) {
    *t = type_lookup(dt);
    return *t != nullptr;
}

// ERR_BUFFER unless the bytes [p + lo, p + hi) lie in memory the GPU can
// access: device memory (hipMalloc, managed memory) or, where host_ok (for
// statuses), pinned host memory -- never pageable host memory, which is
// what a host program would pass by mistake (the GPU example of §6 sends a
// malloc'ed buffer).  When HIP knows the allocation's range, the bytes must
// lie inside it.  HIP is asked once per allocation and stream; the range is
// then kept in the stream's cache.  The check cannot see frees: a range
// freed and reused for other memory while the stream lives passes as the
// allocation it was.
int check_buf(StreamObj *st, const void *p, int64_t lo, int64_t hi, bool host_ok) {
    if (hi <= lo) return MPIXS_SUCCESS;
    if (!p) return MPIXS_ERR_BUFFER;
    const uintptr_t a = uintptr_t(p) + uintptr_t(lo);
    const uintptr_t b = uintptr_t(p) + uintptr_t(hi);
    if (b < a) return MPIXS_ERR_BUFFER;
    if (st) {
        const BufCache &c = st->bufs;
        for (int i = 0; i < BufCache::N; ++i)
            if (c.hi[i] && a >= c.lo[i] && b <= c.hi[i] && (host_ok || !c.host[i]))
                return MPIXS_SUCCESS;
    }
    hipPointerAttribute_t at;
    std::memset(&at, 0, sizeof(at));
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();   // unknown to HIP: pageable host memory
        return MPIXS_ERR_BUFFER;
    }
    bool host = false;
    switch (at.type) {
    case hipMemoryTypeDevice:
    case hipMemoryTypeManaged:
    case hipMemoryTypeUnified: break;
    case hipMemoryTypeHost: host = true; break;
    default: return MPIXS_ERR_BUFFER;
    }
    if (host && !host_ok) return MPIXS_ERR_BUFFER;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void *>(p)) != hipSuccess || !base) {
        (void)hipGetLastError();   // range unknown: accepted, not cached
        return MPIXS_SUCCESS;
    }
    const uintptr_t blo = uintptr_t(base), bhi = blo + size;
    if (a < blo || b > bhi) return MPIXS_ERR_BUFFER;
    if (st) {
        BufCache &c = st->bufs;
        c.lo[c.next] = blo;
        c.hi[c.next] = bhi;
        c.host[c.next] = host;
        c.next = (c.next + 1) % BufCache::N;
    }
    return MPIXS_SUCCESS;
}

// Byte span [lo, hi) that `count` elements of a type touch from a buffer.
void type_span(const TypeObj *t, int count, int64_t *lo, int64_t *hi) {
    if (count <= 0 || t->L.size == 0) {
        *lo = *hi = 0;
        return;
    }
    *lo = t->L.lb;
    *hi = int64_t(count - 1) * t->L.extent + t->L.ub;
}

// Argument checks in a fixed order: communicator, count, datatype, peer,
// tag, overlapping receive type, the library's size limit, buffer.
int check_p2p(mpixs_comm_s *c, const void *buf, int count, mpixs_datatype dt, int peer, int tag,
              bool recv, const TypeObj **t) {
    if (!c || !c->sh) return MPIXS_ERR_COMM;
    if (!c->stream || !c->stream->gpu) return MPIXS_ERR_COMM;
    if (count < 0) return MPIXS_ERR_COUNT;
    if (!type_ok(dt, t)) return MPIXS_ERR_TYPE;
    const bool wild = recv && c->sh->w->cfg.matching == 1;
    if (!(wild && peer == MPIXS_ANY_SOURCE) && (peer < 0 || peer >= c->sh->size))
        return MPIXS_ERR_RANK;
    if (!(wild && tag == MPIXS_ANY_TAG) && tag < 0) return MPIXS_ERR_TAG;
    if (recv && count > 0 && (*t)->L.overlap) return MPIXS_ERR_TYPE;
    const int64_t bytes = int64_t(count) * (*t)->L.size;
    if (!(*t)->L.dense() && bytes >= (int64_t(1) << 32)) return MPIXS_ERR_COUNT;
    if (bytes > 0) {
        int64_t lo, hi;
        type_span(*t, count, &lo, &hi);
        const int rc = check_buf(c->stream, buf, lo, hi, false);
        if (rc) return rc;
    }
    if (c->sh->w->aborted.load()) return MPIXS_ERR_ABORTED;
    return MPIXS_SUCCESS;
}

// First side: wait (host) for the second side's copy launch, then make the
// stream wait for done >= k+1.  For a receive, the wait kernel writes the
// status and the sticky error.
int complete_first(World *w, StreamObj *st, Channel *ch, Rec *rec, uint64_t k, int side,
                   mpixs_status *status) {
    int rc = host_wait(w, &rec->copy_enq, [&] { return rec->copy_enq.load(std::memory_order_acquire) != 0; });
    if (rc) return rc;
    WaitArgs a = wait_one(&rec->d->done, rec->dv);
    if (side == 1) {
        a.status = status;
        a.st = rec->st;
    }
    const bool rel = want_release(ch, rec, k);
    if (rel) {
        a.rel_base = w->h_rel;
        a.rel_idx[0] = rec->didx + 1;
    }
    rc = do_wait(w, st, a, MPIXS_TRACE_COMPLETE);
    if (!rc && rel) note_release(w, ch, rec, k);
    rec_release(ch, rec);
    return rc;
}

// Eager send (a blocking send that arrives first, of at most
// eager_max_bytes): pack message k into device staging on the sender's
// stream; the pack's last workgroup publishes ready[0] (an empty message only
// posts it).  Returns false, having done nothing, when the send must take the
// rendezvous instead (too large, staging full, or eager messages already hold
// half of the matching table).  Caller holds what orders the record (the
// channel's lock, or sole ownership of a fresh channel).
bool eager_try(World *w, StreamObj *st, Rec *rec, const Side &me, int *rc) {
    *rc = MPIXS_SUCCESS;
    if (me.bytes > int64_t(w->cfg.eager_max_bytes) ||
        w->eager_held.load(std::memory_order_relaxed) >= int64_t(w->chan_cap / 2))
        return false;
    uint8_t *stage = nullptr;
    int flag = -1;
    if (me.bytes > 0 && !stage_alloc(w, size_t(me.bytes), &stage, &flag)) return false;
    if (stage) {
        StatusVal pv{};
        pv.count_bytes = me.bytes;
        *rc = do_copy(w, st, me, stage_side(stage, me.bytes, me.rank), pv, nullptr, 0,
                      &rec->d->ready[0], rec->dv, nullptr, false);
    } else {
        *rc = do_post(w, st, &rec->d->ready[0], rec->dv);
    }
    if (*rc) {
        if (stage) stage_drop(w, flag);
        return true;
    }
    rec->eager = true;
    rec->stage = stage;
    rec->stage_flag = flag;
    w->eager_held.fetch_add(1, std::memory_order_relaxed);
    w->n_eager.fetch_add(1, std::memory_order_relaxed);
    return true;
}

// The receive of an eager send, on the receiver's stream: copy from staging
// once the pack has published ready, free the staging slot and, when the
// channel is quiescent, release its block (this copy is its last device use).
int eager_copy(World *w, StreamObj *st, Channel *ch, Rec *rec, uint64_t k, const StatusVal &sv,
               void *status) {
    w->eager_held.fetch_sub(1, std::memory_order_relaxed);
    CopyExtra x;
    if (rec->stage) x.host_flag = &w->stage.flags[rec->stage_flag];
    const bool rel = want_release(ch, rec, k);
    if (rel) {
        x.rel_word = &w->h_rel[rec->didx];
        x.rel_val = rec->dv;
    }
    const Side &S = rec->s;
    const int rc = do_copy(w, st, rec->stage ? stage_side(rec->stage, S.bytes, S.rank) : S, rec->r,
                           sv, &rec->d->ready[0], rec->dv, &rec->d->done, rec->dv, status, true, &x);
    if (rc && rec->stage) stage_drop(w, rec->stage_flag);
    else if (!rc && rel) note_release(w, ch, rec, k);
    return rc;
}

// Ordered-queue matching (§2.1 with wildcards): a send meets the earliest
// posted receive of its destination that accepts (source, tag); a receive
// meets the earliest enqueued send that it accepts; otherwise the operation
// waits in its destination's queue.  "Earliest" is host enqueue order, the
// order in which the enqueue calls reach the library, which keeps MPI's
// non-overtaking rule for each sender and makes a wildcard receive take the
// first matching message enqueued.  Every message gets its own one-message
// channel; the first of the pair posts ready on it and the second copies,
// exactly as on a sequence channel with k = 0.
int p2p_queue(mpixs_comm_s *c, int side, const void *buf, int count, const TypeObj *t, int peer,
              int tag, mpixs_status *status, mpixs_request *req, StreamObj *st, int my_idx,
              int peer_idx) {
    World *w = c->sh->w;
    CommShared *sh = c->sh;
    const int me = c->rank;
    // the destination endpoint's queue
    const int ep = side == 0 ? (sh->multiplex ? sh->ep_base[size_t(peer)] + peer_idx : peer)
                             : (sh->multiplex ? sh->ep_base[size_t(me)] + my_idx : me);
    MatchQueue &q = sh->mq[size_t(ep)];
    Side mine;
    mine.buf = buf;
    mine.count = count;
    mine.t = t;
    mine.bytes = int64_t(count) * t->L.size;
    mine.st = st;
    mine.rank = me;
    mine.idx = my_idx;
    mpixs_request_s *r = req ? new mpixs_request_s() : nullptr;
    if (r) r->stream = st;
    std::unique_lock<std::mutex> lk(q.mu);
    QOp partner;
    bool found = false;
    if (side == 0) {
        for (auto it = q.posted.begin(); it != q.posted.end(); ++it) {
            if ((it->src == MPIXS_ANY_SOURCE || it->src == me) &&
                (it->src_idx == MPIXS_ANY_INDEX || it->src_idx == my_idx) &&
                (it->tag == MPIXS_ANY_TAG || it->tag == tag)) {
                partner = *it;
                q.posted.erase(it);
                found = true;
                break;
            }
        }
    } else {
        for (auto it = q.unexpected.begin(); it != q.unexpected.end(); ++it) {
            if ((peer == MPIXS_ANY_SOURCE || it->src == peer) &&
                (peer_idx == MPIXS_ANY_INDEX || it->src_idx == peer_idx) &&
                (tag == MPIXS_ANY_TAG || it->tag == tag)) {
                partner = *it;
                q.unexpected.erase(it);
                found = true;
                break;
            }
        }
    }
    int rc = MPIXS_SUCCESS;
    if (found) {
        lk.unlock();
        // second of the pair: the partner publishes its operation in the
        // queue before it enqueues its ready post (so that launches happen
        // outside the queue lock); wait for that post to be enqueued, so the
        // device wait below never precedes its producer
        Channel *ch = partner.ch;
        Rec *rec = partner.rec;
        const uint32_t other = side == 0 ? ARR_R : ARR_S;
        rc = host_wait(w, &rec->arrived, [&] {
            return (rec->arrived.load(std::memory_order_acquire) & other) != 0;
        });
        if (rc) {
            delete r;
            return rc;
        }
        {
            std::lock_guard<std::mutex> g(ch->mu);
            (side == 0 ? rec->s : rec->r) = mine;
        }
        const int mtag = side == 0 ? tag : partner.tag;
        const StatusVal sv = match_status(rec->s, rec->r, mtag);
        const bool recv_here = side == 1;
        if (rec->eager)
            rc = eager_copy(w, st, ch, rec, 0, sv, req ? nullptr : static_cast<void *>(status));
        else
            rc = do_copy(w, st, rec->s, rec->r, sv, &rec->d->ready[1 - side], rec->dv, &rec->d->done,
                         rec->dv, (recv_here && !req) ? static_cast<void *>(status) : nullptr,
                         recv_here);
        rec->st = sv;
        rec->copy_enq.store(1, std::memory_order_release);
        host_notify(&rec->copy_enq);
        rec_release(ch, rec);
        if (r) {
            r->comm = c;
            r->side = side;
            r->second = true;
            r->st = sv;
            r->k = 0;
            c->pending.fetch_add(1);
            *req = r;
        }
        return rc;
    }
    // first of the pair: a fresh one-message channel, published in the queue
    // and then posted outside the lock (a partner waits on the host until
    // the post is enqueued)
    Channel *ch = new Channel();
    ch->priv = true;
    rc = attach_block(w, ch, 0);
    if (rc) {
        delete ch;
        delete r;
        return rc;
    }
    Rec *rec = ch->at(0);
    set_rec_block(ch, rec, 0);
    (side == 0 ? rec->s : rec->r) = mine;
    QOp op;
    op.ch = ch;
    op.rec = rec;
    op.src = side == 0 ? me : peer;
    op.src_idx = side == 0 ? my_idx : peer_idx;
    op.tag = tag;
    (side == 0 ? q.unexpected : q.posted).push_back(op);
    lk.unlock();
    // a partner reads the record only once `arrived` shows this side's post
    const bool eager = side == 0 && !req && eager_try(w, st, rec, mine, &rc);
    if (!eager) rc = do_post(w, st, &rec->d->ready[side], rec->dv);
    rec->arrived.fetch_or(side == 0 ? ARR_S : ARR_R, std::memory_order_release);
    host_notify(&rec->arrived);
    if (rc) {
        // the operation is already visible to partners: stop the world
        // rather than leave one waiting for a post that never comes
        mpixs_world_abort(reinterpret_cast<mpixs_world>(w));
        delete r;
        return rc;
    }
    if (eager) {
        rec_release(ch, rec);   // nothing of the send waits for its receive
        return MPIXS_SUCCESS;
    }
    if (!r) return complete_first(w, st, ch, rec, 0, side, status);
    r->comm = c;
    r->ch = ch;
    r->rec = rec;
    r->k = 0;
    r->side = side;
    r->second = false;
    c->pending.fetch_add(1);
    *req = r;
    return MPIXS_SUCCESS;
}

int p2p(mpixs_comm_s *c, int side, const void *buf, int count, mpixs_datatype dt, int peer,
        int tag, mpixs_status *status, mpixs_request *req) {
    const TypeObj *t = nullptr;
    int rc = check_p2p(c, buf, count, dt, peer, tag, side == 1, &t);
    if (!rc && status) rc = check_buf(c->stream, status, 0, sizeof(mpixs_status), true);
    if (rc) return rc;
    World *w = c->sh->w;
    StreamObj *st = c->stream;
    if (c->in_group && side == 1 && peer == MPIXS_ANY_SOURCE) return MPIXS_ERR_RANK;
    if (c->in_group && side == 1 && tag == MPIXS_ANY_TAG) return MPIXS_ERR_TAG;
    if (!c->in_group && w->cfg.matching == 1)
        return p2p_queue(c, side, buf, count, t, peer, tag, status, req, st, 0, 0);
    if (c->in_group) {
        // recorded; mpixs_group_end enqueues it
        GOp g;
        g.kind = side;
        g.peer = peer;
        g.tag = tag;
        g.side.buf = buf;
        g.side.count = count;
        g.side.t = t;
        g.side.bytes = int64_t(count) * t->L.size;
        g.side.st = st;
        g.side.rank = c->rank;
        g.status = (side == 1 && !req) ? static_cast<void *>(status) : nullptr;
        if (req) {
            mpixs_request_s *r = new mpixs_request_s();
            r->comm = c;
            r->side = side;
            r->grouped = true;
            r->gop = c->gops.size();
            g.req = r;
            c->pending.fetch_add(1);
            *req = r;
        }
        c->gops.push_back(g);
        return MPIXS_SUCCESS;
    }
    const int src = side == 0 ? c->rank : peer;
    const int dst = side == 0 ? peer : c->rank;
    Channel *ch = get_channel(c, src, dst, tag, false);
    if (!ch) return MPIXS_ERR_NOMEM;
    mpixs_request_s *r = nullptr;
    if (req) {
        r = new mpixs_request_s();
        r->stream = st;
    }
    Side me;
    me.buf = buf;
    me.count = count;
    me.t = t;
    me.bytes = int64_t(count) * t->L.size;
    me.st = st;
    me.rank = c->rank;
    const uint32_t mine = side == 0 ? ARR_S : ARR_R;
    const uint32_t other = side == 0 ? ARR_R : ARR_S;

    ch->mu.lock();
    const uint64_t k = ch->seq[side];
    if (!ch->d) {
        rc = attach_block(w, ch, k);
        if (rc) {
            ch->mu.unlock();
            delete r;
            return rc;
        }
    }
    ch->seq[side] = k + 1;
    Rec *rec = ch->at(k);
    set_rec_block(ch, rec, k);
    (side == 0 ? rec->s : rec->r) = me;
    const bool second = (rec->arrived.load(std::memory_order_relaxed) & other) != 0;
    if (second) {
        ch->mu.unlock();
        const Side &S = rec->s;
        const Side &R = rec->r;
        const StatusVal sv = match_status(S, R, tag);
        const bool recv_here = side == 1;
        if (rec->eager) {
            rc = eager_copy(w, st, ch, rec, k, sv, req ? nullptr : static_cast<void *>(status));
        } else {
            rc = do_copy(w, st, S, R, sv, &rec->d->ready[1 - side], rec->dv, &rec->d->done, rec->dv,
                         (recv_here && !req) ? static_cast<void *>(status) : nullptr, recv_here);
        }
        rec->st = sv;
        rec->copy_enq.store(1, std::memory_order_release);
        host_notify(&rec->copy_enq);
        rec_release(ch, rec);
        if (r) {
            r->comm = c;
            r->side = side;
            r->second = true;
            r->st = sv;
            r->k = k;
            c->pending.fetch_add(1);
            *req = r;
        }
        return rc;
    }
    // a blocking send that arrives first: eager when it can be (a
    // nonblocking send keeps the rendezvous: its call returns at once anyway,
    // and a post costs less than a pack)
    if (side == 0 && !req && eager_try(w, st, rec, me, &rc)) {
        if (rc) {
            ch->seq[side] = k;   // nothing was enqueued: the call has no effect
            ch->mu.unlock();
            return rc;
        }
        rec->arrived.fetch_or(mine, std::memory_order_release);
        host_notify(&rec->arrived);
        ch->mu.unlock();
        rec_release(ch, rec);   // nothing of the send waits for its receive
        return MPIXS_SUCCESS;
    }
    rc = do_post(w, st, &rec->d->ready[side], rec->dv);
    rec->arrived.fetch_or(mine, std::memory_order_release);
    host_notify(&rec->arrived);
    ch->mu.unlock();
    if (rc) {
        delete r;
        return rc;
    }
    if (!r) return complete_first(w, st, ch, rec, k, side, status);
    r->comm = c;
    r->ch = ch;
    r->rec = rec;
    r->k = k;
    r->side = side;
    r->second = false;
    c->pending.fetch_add(1);
    *req = r;
    return MPIXS_SUCCESS;
}

// ----------------------------------------------------------------- waits
int wait_many(int n, mpixs_request *reqs, mpixs_status *statuses, bool array_status) {
    if (n < 0) return MPIXS_ERR_COUNT;
    if (n == 0) return MPIXS_SUCCESS;
    if (!reqs) return MPIXS_ERR_REQUEST;
    StreamObj *st = nullptr;
    for (int i = 0; i < n; ++i) {
        mpixs_request_s *r = reqs[i];
        if (!r || !r->comm) return MPIXS_ERR_REQUEST;
        StreamObj *rs = r->stream ? r->stream : r->comm->stream;
        if (st && rs != st) return MPIXS_ERR_STREAM;
        st = rs;
    }
    if (statuses) {
        const int rc = check_buf(st, statuses, 0,
                                 int64_t(array_status ? n : 1) * int64_t(sizeof(mpixs_status)), true);
        if (rc) return rc;
    }
    World *w = reqs[0]->comm->sh->w;
    int rc = MPIXS_SUCCESS;
    // grouped requests: inside their group the status pointer is recorded;
    // after it the transfer is complete in stream order and only the status
    // remains to be written
    for (int i = 0; i < n && !rc; ++i) {
        mpixs_request_s *r = reqs[i];
        if (!r->grouped) continue;
        mpixs_status *status = statuses ? (array_status ? &statuses[i] : statuses) : nullptr;
        mpixs_comm_s *c = r->comm;
        if (c->in_group && r->gop < c->gops.size() && c->gops[r->gop].req == r) {
            c->gops[r->gop].req = nullptr;
            if (r->side == 1) c->gops[r->gop].status = status;
        } else if (r->side == 1 && status) {
            WaitArgs s;
            std::memset(&s, 0, sizeof(s));
            s.status = status;
            s.st = r->st;
            rc = do_wait(w, st, s, 0);
        }
    }
    // first-side requests: host-wait for each copy launch, then one wait
    // kernel per 64 of them; second-side receives only need their status.
    WaitArgs a;
    std::memset(&a, 0, sizeof(a));
    std::vector<std::pair<int, mpixs_request_s *>> batch;
    auto flush = [&]() -> int {
        if (a.n == 0) return MPIXS_SUCCESS;
        int r2 = do_wait(w, st, a, MPIXS_TRACE_COMPLETE);
        for (size_t j = 0; j < batch.size(); ++j) {
            mpixs_request_s *q = batch[j].second;
            if (!q->rec) continue;
            if (!r2 && a.rel_idx[j]) note_release(w, q->ch, q->rec, q->k);
            rec_release(q->ch, q->rec);
        }
        std::memset(&a, 0, sizeof(a));
        batch.clear();
        return r2;
    };
    // one first-side wait lane, releasing the message's block when it is
    // the block's last device use
    auto lane_of = [&](WaitArgs &x, mpixs_request_s *q) -> bool {
        x.ptr[x.n] = &q->rec->d->done;
        x.target[x.n] = q->rec->dv;
        const bool rel = want_release(q->ch, q->rec, q->k);
        if (rel) {
            x.rel_base = w->h_rel;
            x.rel_idx[x.n] = q->rec->didx + 1;
        }
        x.n++;
        return rel;
    };
    for (int i = 0; i < n && !rc; ++i) {
        mpixs_request_s *r = reqs[i];
        mpixs_status *status = statuses ? (array_status ? &statuses[i] : statuses) : nullptr;
        if (r->grouped) continue;
        if (r->second) {
            if (r->side == 1 && status) {
                // the copy ran on this stream; only the status remains
                WaitArgs s;
                std::memset(&s, 0, sizeof(s));
                s.status = status;
                s.st = r->st;
                rc = flush();
                if (!rc) rc = do_wait(w, st, s, 0);
            }
            continue;
        }
        rc = host_wait(w, &r->rec->copy_enq, [&] { return r->rec->copy_enq.load(std::memory_order_acquire) != 0; });
        if (rc) break;
        if (r->side == 1 && (status || r->rec->st.error)) {
            // a status (or a sticky error) per wait kernel
            rc = flush();
            if (rc) break;
            WaitArgs s;
            std::memset(&s, 0, sizeof(s));
            const bool rel = lane_of(s, r);
            s.status = status;
            s.st = r->rec->st;
            rc = do_wait(w, st, s, MPIXS_TRACE_COMPLETE);
            if (!rc && rel) note_release(w, r->ch, r->rec, r->k);
            rec_release(r->ch, r->rec);
            r->rec = nullptr;
            continue;
        }
        lane_of(a, r);
        batch.emplace_back(i, r);
        if (a.n == 64) rc = flush();
    }
    if (!rc) rc = flush();
    for (int i = 0; i < n; ++i) {
        mpixs_request_s *r = reqs[i];
        r->comm->pending.fetch_sub(1);
        delete r;
        reqs[i] = nullptr;
    }
    return rc;
}

// -------------------------------------------------------------- allreduce
int check_allreduce(mpixs_comm_s *c, const void *sendbuf, void *recvbuf, int count,
                    mpixs_datatype dt, mpixs_op op, bool need_stream) {
    if (!c || !c->sh) return MPIXS_ERR_COMM;
    if (need_stream && (!c->stream || !c->stream->gpu)) return MPIXS_ERR_COMM;
    if (count < 0) return MPIXS_ERR_COUNT;
    if (dt != MPIXS_INT32 && dt != MPIXS_INT64 && dt != MPIXS_FLOAT32 && dt != MPIXS_FLOAT64)
        return MPIXS_ERR_TYPE;
    if (op < MPIXS_SUM || op > MPIXS_MAX) return MPIXS_ERR_OP;
    if (c->sh->size > 64) return MPIXS_ERR_COMM;
    if (count > 0) {
        const int64_t bytes = int64_t(count) * basic_size(dt);
        int rc = sendbuf == MPIXS_IN_PLACE ? MPIXS_SUCCESS
                                           : check_buf(c->stream, sendbuf, 0, bytes, false);
        if (!rc) rc = check_buf(c->stream, recvbuf, 0, bytes, false);
        if (rc) return rc;
    }
    if (c->sh->w->aborted.load()) return MPIXS_ERR_ABORTED;
    return MPIXS_SUCCESS;
}

int do_reduce(World *w, StreamObj *on, CollRec *rec, int n, int me, const uint64_t *arrive,
              uint64_t target, uint64_t *done_ptr, uint64_t done_val) {
    ReduceArgs a;
    std::memset(&a, 0, sizeof(a));
    bool vec = true;
    for (int q = 0; q < n; ++q) {
        a.in[q] = rec->in[q];
        a.out[q] = rec->out[q];
        vec = vec && (reinterpret_cast<uintptr_t>(rec->in[q]) % 16 == 0) &&
              (reinterpret_cast<uintptr_t>(rec->out[q]) % 16 == 0);
    }
    a.n = n;
    a.me_rank = me;
    a.count = uint64_t(rec->count);
    const int es = basic_size(rec->dtype);
    const int64_t bytes = int64_t(rec->count) * es;
    const bool fuse = w->cfg.fuse_max_bytes >= 0 && bytes * n <= int64_t(w->cfg.fuse_max_bytes);
    const uint64_t per_thread = vec ? uint64_t(16 / es) : 1;
    const uint64_t work = (a.count + per_thread - 1) / per_thread;
    const uint64_t nchunks = std::max<uint64_t>(1, (work + reduce_threads() - 1) / reduce_threads());
    int rc = MPIXS_SUCCESS;
    a.ctl = ctl_of(w);
    a.me = on->dev;
    hipEvent_t e0 = nullptr;
    if (fuse) {
        const uint64_t nwg = std::min<uint64_t>(nchunks, kFusedMaxWG);
        if (arrive && n > 1) {
            a.arrive = arrive;
            a.arrive_target = target;
        }
        a.done_ptr = done_ptr;
        a.done_val = done_val;
        a.ticket_last = on->tickets + nwg - 1;
        a.trace = trace_kind(w, 1);
        if (profile_on(w)) prof_begin(w, on->hs, &e0);
        rc = gpu_err(launch_reduce(on->hs, a, rec->dtype, rec->op, vec, int(nwg), true));
        if (profile_on(w)) prof_end(w, on->hs, e0, 1);
        if (rc) return rc;
        if (nwg > 1) on->tickets += nwg;
    } else {
        if (arrive && n > 1) {
            WaitArgs wa;
            std::memset(&wa, 0, sizeof(wa));
            for (int q = 0; q < n; ++q) {
                if (q == me) continue;
                wa.ptr[wa.n] = arrive + 16 * q;
                wa.target[wa.n] = target;
                wa.n++;
            }
            rc = do_wait(w, on, wa, MPIXS_TRACE_MATCH);
            if (rc) return rc;
        }
        const bool fixed = vec && reduce_fixed_ok(n);
        const uint64_t per_wg = fixed ? uint64_t(reduce_fixed_units()) : 1;
        const uint64_t nwg = std::min<uint64_t>((nchunks + per_wg - 1) / per_wg, uint64_t(1) << 22);
        if (profile_on(w)) prof_begin(w, on->hs, &e0);
        rc = gpu_err(fixed ? launch_reduce_fixed(on->hs, a, rec->dtype, rec->op, int(nwg))
                           : launch_reduce(on->hs, a, rec->dtype, rec->op, vec, int(nwg), false));
        if (profile_on(w)) prof_end(w, on->hs, e0, 1);
        if (rc) return rc;
        if (done_ptr) {
            SignalArgs sg;
            std::memset(&sg, 0, sizeof(sg));
            sg.done_ptr = done_ptr;
            sg.done_val = done_val;
            sg.me = on->dev;
            sg.trace = trace_kind(w, 1);
            rc = gpu_err(launch_signal(on->hs, sg));
            if (rc) return rc;
            w->n_post.fetch_add(1, std::memory_order_relaxed);
        }
    }
    w->n_reduce.fetch_add(1, std::memory_order_relaxed);
    w->bytes_reduced.fetch_add(uint64_t(2 * bytes * n), std::memory_order_relaxed);
    return MPIXS_SUCCESS;
}

// A grouped allreduce: the split reduce kernel over all ranks' buffers, run
// on the launching rank's stream after the group's wait (and batch kernel).
RedPlan plan_red(World *w, const std::vector<const GOp *> &calls, StreamObj *on) {
    RedPlan r;
    const int n = int(calls.size());
    bool vec = true;
    for (int q = 0; q < n; ++q) {
        r.a.in[q] = calls[size_t(q)]->red_in;
        r.a.out[q] = calls[size_t(q)]->red_out;
        vec = vec && (reinterpret_cast<uintptr_t>(r.a.in[q]) % 16 == 0) &&
              (reinterpret_cast<uintptr_t>(r.a.out[q]) % 16 == 0);
    }
    const GOp &c0 = *calls[0];
    r.a.n = n;
    r.a.me_rank = -1;
    r.a.count = uint64_t(c0.red_count);
    r.a.ctl = ctl_of(w);
    r.a.me = on->dev;
    r.dtype = c0.red_dtype;
    r.op = c0.red_op;
    const int es = basic_size(r.dtype);
    const uint64_t per_thread = vec ? uint64_t(16 / es) : 1;
    const uint64_t work = (r.a.count + per_thread - 1) / per_thread;
    const uint64_t nchunks = std::max<uint64_t>(1, (work + reduce_threads() - 1) / reduce_threads());
    r.vec = vec;
    r.fixed = vec && reduce_fixed_ok(n);
    const uint64_t per_wg = r.fixed ? uint64_t(reduce_fixed_units()) : 1;
    r.nwg = int(std::min<uint64_t>((nchunks + per_wg - 1) / per_wg, uint64_t(1) << 22));
    r.bytes = uint64_t(2) * uint64_t(c0.red_count) * uint64_t(es) * uint64_t(n);
    return r;
}

int launch_red(World *w, hipStream_t s, const RedPlan &r) {
    if (r.a.count == 0) return MPIXS_SUCCESS;
    const int rc = gpu_err(r.fixed ? launch_reduce_fixed(s, r.a, r.dtype, r.op, r.nwg)
                                   : launch_reduce(s, r.a, r.dtype, r.op, r.vec, r.nwg, false));
    if (!rc && w) {
        w->n_reduce.fetch_add(1, std::memory_order_relaxed);
        w->bytes_reduced.fetch_add(r.bytes, std::memory_order_relaxed);
    }
    return rc;
}

// Merge a group's allreduces into one launch when they are all small, of
// one type and operator, and no byte of any of their buffers belongs to two
// of them; otherwise m.on stays false and they run one by one, in order.
// Zero-count allreduces do nothing either way and are left out.
constexpr uint64_t kMultiRedMaxBytes = uint64_t(64) << 20;   // per allreduce, all ranks' input
constexpr uint64_t kMultiRedMaxWG = uint64_t(1) << 20;
// merged launches moving at least this much use nontemporal accesses
constexpr uint64_t kMultiRedNtBytes = uint64_t(64) << 20;

void plan_multi_red(const std::vector<RedPlan> &reds, MultiRedPlan &m) {
    m.on = false;
    m.nt = false;
    m.desc.clear();
    m.ptrs.clear();
    m.bytes = 0;
    m.ninst = 0;
    m.nwg = 0;
    if (reds.size() < 2) return;
    struct Span {
        uintptr_t lo, hi;
        uint32_t inst;
    };
    std::vector<Span> spans;
    std::vector<uint64_t> units;       // per merged allreduce
    for (size_t i = 0; i < reds.size(); ++i) {
        const RedPlan &r = reds[i];
        if (r.dtype != reds[0].dtype || r.op != reds[0].op) return;
        if (r.a.count == 0) continue;
        if (r.a.n < 1 || r.a.n > 64) return;
        const uint64_t es = uint64_t(basic_size(r.dtype));
        const uint64_t len = r.a.count * es;
        if (len * uint64_t(r.a.n) > kMultiRedMaxBytes) return;
        units.push_back(r.vec ? std::max<uint64_t>(1, r.a.count / (16 / es)) : r.a.count);
        MultiRedDesc d{};
        d.count = r.a.count;
        d.ptr = uint32_t(m.ptrs.size());
        d.n = uint32_t(r.a.n);
        d.vec = r.vec ? 1u : 0u;
        for (int q = 0; q < r.a.n; ++q) {
            m.ptrs.push_back(r.a.in[q]);
            spans.push_back(Span{uintptr_t(r.a.in[q]), uintptr_t(r.a.in[q]) + len, uint32_t(i)});
        }
        for (int q = 0; q < r.a.n; ++q) {
            m.ptrs.push_back(r.a.out[q]);
            spans.push_back(Span{uintptr_t(r.a.out[q]), uintptr_t(r.a.out[q]) + len, uint32_t(i)});
        }
        m.desc.push_back(d);
        m.bytes += r.bytes;
    }
    if (m.desc.size() < 2) return;
    // workgroups: chunks of reduce_multi_units(nt) vectors (or elements)
    m.nt = m.bytes >= kMultiRedNtBytes;
    const uint64_t per = uint64_t(reduce_multi_units(m.nt));
    uint64_t wg = 0;
    for (size_t i = 0; i < m.desc.size(); ++i) {
        m.desc[i].first_wg = uint32_t(wg);
        wg += (units[i] + per - 1) / per;
        if (wg > kMultiRedMaxWG) return;
    }
    // Sweep the spans by start, keeping the farthest end seen and its
    // allreduce.  The first span (in this order) that overlaps a span of
    // another allreduce always starts before that farthest end, and the end
    // belongs to another allreduce (were it its own, that span and the
    // overlapped one would both hold this start and overlap earlier).
    std::sort(spans.begin(), spans.end(),
              [](const Span &x, const Span &y) { return x.lo < y.lo || (x.lo == y.lo && x.hi < y.hi); });
    uintptr_t end = 0;
    uint32_t owner = 0;
    bool any = false;
    for (const Span &sp : spans) {
        if (any && sp.lo < end && sp.inst != owner) return;
        if (!any || sp.hi > end) {
            end = sp.hi;
            owner = sp.inst;
            any = true;
        }
    }
    m.dtype = reds[0].dtype;
    m.op = reds[0].op;
    m.nwg = int(wg);
    m.ninst = uint32_t(m.desc.size());
    m.on = true;
}

// Counters of a run whose allreduces a graph replay launched.
void count_reds(World *w, const std::vector<RedPlan> &reds, const MultiRedPlan &m) {
    if (m.on) {
        w->n_reduce.fetch_add(1, std::memory_order_relaxed);
        w->reds_merged.fetch_add(m.ninst, std::memory_order_relaxed);
        w->bytes_reduced.fetch_add(m.bytes, std::memory_order_relaxed);
        return;
    }
    for (const RedPlan &r : reds)
        if (r.a.count > 0) {
            w->n_reduce.fetch_add(1, std::memory_order_relaxed);
            w->bytes_reduced.fetch_add(r.bytes, std::memory_order_relaxed);
        }
}

// The group's allreduces on stream s (w may be null: graph capture).
int launch_reds(World *w, hipStream_t s, const std::vector<RedPlan> &reds, const MultiRedPlan &m,
                const MultiRedArgs &ma) {
    if (m.on) {
        const int rc = gpu_err(launch_reduce_multi(s, ma, m.dtype, m.op, m.nwg, m.nt));
        if (!rc && w) {
            w->n_reduce.fetch_add(1, std::memory_order_relaxed);
            w->reds_merged.fetch_add(m.ninst, std::memory_order_relaxed);
            w->bytes_reduced.fetch_add(m.bytes, std::memory_order_relaxed);
        }
        return rc;
    }
    for (const RedPlan &r : reds) {
        const int rc = launch_red(w, s, r);
        if (rc) return rc;
    }
    return MPIXS_SUCCESS;
}

CollRec *coll_at(std::deque<CollRec *> &q, uint64_t &base, uint64_t k, int size) {
    while (base + q.size() <= k) {
        CollRec *r = new CollRec();
        r->refs.store(size);
        q.push_back(r);
    }
    return q[k - base];
}

void coll_collect(std::deque<CollRec *> &q, uint64_t &base) {
    while (!q.empty() && q.front()->refs.load() == 0) {
        delete q.front();
        q.pop_front();
        ++base;
    }
}

// ------------------------------------------------------------- batches
// Reserve `bytes` of the host-pinned descriptor arena and a completion flag.
// Entries are recycled in order once their batch's signal kernel has set
// the flag; if the arena is full the host waits for the oldest batch, which
// was enqueued after everything it waits for and so always finishes.
int arena_alloc(World *w, size_t bytes, size_t *off, int *flag) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes > w->arena_bytes) return MPIXS_ERR_NOMEM;
    std::unique_lock<std::mutex> g(w->arena_mu);
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        while (!w->arena_live.empty() &&
               __atomic_load_n(&w->h_flags[w->arena_live.front().flag], __ATOMIC_ACQUIRE) == 1) {
            w->free_flags.push_back(w->arena_live.front().flag);
            w->arena_live.pop_front();
        }
        if (w->arena_live.empty()) w->arena_head = 0;
        bool ok = false;
        size_t at = 0;
        if (!w->free_flags.empty()) {
            if (w->arena_live.empty()) {
                ok = true;
                at = 0;
            } else {
                const size_t tail = w->arena_live.front().off;
                if (w->arena_head >= tail) {
                    if (w->arena_head + bytes <= w->arena_bytes) {
                        ok = true;
                        at = w->arena_head;
                    } else if (bytes < tail) {
                        ok = true;
                        at = 0;
                    }
                } else if (w->arena_head + bytes < tail) {
                    ok = true;
                    at = w->arena_head;
                }
            }
        }
        if (ok) {
            const int f = w->free_flags.back();
            w->free_flags.pop_back();
            __atomic_store_n(&w->h_flags[f], 0u, __ATOMIC_RELEASE);
            w->arena_live.push_back(World::ArenaUse{at, bytes, f});
            w->arena_head = at + bytes;
            *off = at;
            *flag = f;
            return MPIXS_SUCCESS;
        }
        if (w->aborted.load()) return MPIXS_ERR_ABORTED;
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(w->cfg.timeout_ms))
            return MPIXS_ERR_TIMEOUT;
        g.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        g.lock();
    }
}

// Descriptor chunks of a group's plan, and the size from which the waiting
// ranks help with them (below it the wake-ups cost more than they save).
constexpr size_t kPlanChunk = 256;
constexpr size_t kPlanHelpPairs = 2048;

// Take chunks of the group's published planning job until none is left.
void plan_help(GroupRec *rec) {
    for (;;) {
        const size_t c = rec->help_next.fetch_add(1, std::memory_order_relaxed);
        if (c >= rec->help_chunks) return;
        rec->help_fn(c);
        rec->help_done.fetch_add(1, std::memory_order_release);
    }
}

// Where a plan's descriptors and workgroup starts are written: given the
// number of pairs and a bound on the starts, the caller provides both
// arrays (or fails with an error code).
using PlanPlace = std::function<int(size_t npairs, size_t max_starts, BatchDesc **descs,
                                    BatchStart **starts)>;

// Match every rank's recorded operations of a group (the i-th grouped send
// of s to d with tag t pairs with the i-th grouped receive of d from s with
// tag t), plan each copy, and cut the group into tiles: one descriptor per
// message and, per workgroup, the (message, tile) it starts at, written
// where `place` puts them (else into the plan's own arrays).  Fills `a`,
// its descriptor / start pointers aimed at where they were written.
int plan_group(World *w, CommShared *sh, GroupRec *rec, int n, StreamObj *launcher, BatchArgs &a,
               uint64_t *bytes, const PlanPlace *place = nullptr) {
    struct PlanTimer {   // host time of this plan, for the diagnostics counters
        World *w;
        std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
        ~PlanTimer() {
            const auto ns = std::chrono::duration_cast<std::chrono::nanoseconds>(
                std::chrono::steady_clock::now() - t0).count();
            w->plan_ns.fetch_add(uint64_t(ns), std::memory_order_relaxed);
            w->groups_planned.fetch_add(1, std::memory_order_relaxed);
        }
    } timer{w};
    // Matching in two linear passes over flat arrays (no per-channel
    // containers): an open-addressing table numbers the channels in order of
    // first appearance and counts each channel's sends and receives; the
    // second pass lays the sends and the receives out channel by channel in
    // program order, so the i-th send of a channel sits beside its i-th
    // receive.  The arrays belong to the communicator and keep their memory
    // from one instance to the next (instances of a communicator are planned
    // one at a time, under plan_mu).
    PlanScratch &z = sh->plan;
    size_t nops = 0;
    for (int q = 0; q < n; ++q) nops += rec->ops[size_t(q)].size();
    // a matched group has at most nops / 2 channels, so the table is at most
    // half full (and a group of unmatched operations, refused below, still
    // finds a free slot for each of its at most nops channels)
    size_t cap = 16;
    int lg = 4;
    while (cap < nops) {
        cap <<= 1;
        ++lg;
    }
    constexpr uint64_t kEmpty = ~uint64_t(0);   // no channel key has bit 63 set
    z.table.assign(cap, PlanScratch::Slot{kEmpty, 0});
    z.chan_of.resize(nops);
    z.nsend.clear();
    z.nrecv.clear();
    size_t k = 0;
    for (int q = 0; q < n; ++q)
        for (GOp &op : rec->ops[size_t(q)]) {
            if (op.kind == 2) continue;   // allreduces: below
            const uint64_t key = op.kind == 0 ? chan_key(q, op.peer, op.tag) : chan_key(op.peer, q, op.tag);
            // Fibonacci hashing: the product's top lg bits (its low bits
            // depend on the tag alone, which clusters every channel of a tag)
            size_t h = size_t((key * 0x9E3779B97F4A7C15ull) >> (64 - lg));
            while (z.table[h].key != kEmpty && z.table[h].key != key) h = (h + 1) & (cap - 1);
            if (z.table[h].key == kEmpty) {
                z.table[h] = PlanScratch::Slot{key, uint32_t(z.nsend.size())};
                z.nsend.push_back(0);
                z.nrecv.push_back(0);
            }
            const uint32_t c = z.table[h].chan;
            z.chan_of[k++] = c;
            ++(op.kind == 0 ? z.nsend : z.nrecv)[c];
        }
    const size_t nch = z.nsend.size();
    z.first.assign(nch + 1, 0);   // first pair of each channel
    for (size_t c = 0; c < nch; ++c) {
        if (z.nsend[c] != z.nrecv[c]) return MPIXS_ERR_ARG;
        z.first[c + 1] = z.first[c] + z.nsend[c];
    }
    const size_t npairs = z.first[nch];
    z.s_of.resize(npairs);
    z.r_of.resize(npairs);
    z.fill_s.assign(z.first.begin(), z.first.end() - 1);
    z.fill_r = z.fill_s;
    k = 0;
    for (int q = 0; q < n; ++q)
        for (GOp &op : rec->ops[size_t(q)]) {
            if (op.kind == 2) continue;
            const uint32_t c = z.chan_of[k++];
            if (op.kind == 0) z.s_of[z.fill_s[c]++] = &op;
            else z.r_of[z.fill_r[c]++] = &op;
        }
    // allreduces: the i-th grouped allreduce of every rank forms reduction
    // i; ranks must have grouped as many, with equal count, type and op
    z.reds.clear();
    {
        std::vector<std::vector<const GOp *>> per(static_cast<size_t>(n));
        for (int q = 0; q < n; ++q)
            for (const GOp &op : rec->ops[size_t(q)])
                if (op.kind == 2) per[size_t(q)].push_back(&op);
        const size_t m = per[0].size();
        for (int q = 1; q < n; ++q)
            if (per[size_t(q)].size() != m) return MPIXS_ERR_ARG;
        std::vector<const GOp *> calls(static_cast<size_t>(n));
        for (size_t i = 0; i < m; ++i) {
            for (int q = 0; q < n; ++q) {
                const GOp *o = per[size_t(q)][i];
                if (o->red_count != per[0][i]->red_count || o->red_dtype != per[0][i]->red_dtype ||
                    o->red_op != per[0][i]->red_op)
                    return MPIXS_ERR_ARG;
                calls[size_t(q)] = o;
            }
            z.reds.push_back(plan_red(w, calls, launcher));
        }
        plan_multi_red(z.reds, z.mred);
    }
    const uint32_t tile = uint32_t(w->cfg.batch_tile);
    // descriptors and starts go where the caller places them (a launch's
    // pinned arena range, written once), else into the plan's own arrays
    BatchDesc *D = nullptr;
    BatchStart *SB = nullptr;
    z.nstarts = 0;
    if (place && npairs > 0) {
        const int prc = (*place)(npairs, size_t(w->cfg.batch_max_wg), &D, &SB);
        if (prc) return prc;
        z.descs.clear();
    } else {
        z.descs.resize(npairs);
        D = z.descs.data();
    }
    uint64_t total_tiles = 0;
    *bytes = 0;
    // descriptors in chunks of pairs; each chunk's tiles and bytes summed
    // apart (a channel's pairs share its tag, which every send carries)
    const size_t nchunks = (npairs + kPlanChunk - 1) / kPlanChunk;
    z.part.assign(2 * nchunks, 0);
    auto chunk = [D, &z, tile, npairs](size_t c) {
        uint64_t tiles = 0, nbytes = 0;
        const size_t end = std::min(npairs, (c + 1) * kPlanChunk);
        for (size_t i = c * kPlanChunk; i < end; ++i) {
            GOp *S = z.s_of[i];
            GOp *R = z.r_of[i];
            BatchDesc &d = D[i];
            std::memset(&d, 0, sizeof(d));
            d.st = match_status(S->side, R->side, S->tag);
            int wsz = 16;
            uint64_t units = 0;
            plan_copy(S->side, R->side, d.st.count_bytes, &d.src, &d.dst, &wsz, &units, &d.tail);
            d.units = units;
            d.w = uint32_t(wsz);
            const uint64_t tu = uint64_t(tile) * uint64_t(16 / wsz);   // units per tile
            d.ntiles = uint32_t(std::max<uint64_t>(1, (units + tu - 1) / tu));
            d.status = R->status;
            d.rstream = R->side.st->dev;
            if (R->req) R->req->st = d.st;
            tiles += d.ntiles;
            nbytes += uint64_t(d.st.count_bytes);
        }
        z.part[2 * c] = tiles;
        z.part[2 * c + 1] = nbytes;
    };
    if (n > 1 && npairs >= kPlanHelpPairs) {
        // the other ranks wait for this launch on the host: let them take
        // chunks too (those asleep are woken through the launch's key)
        rec->help_fn = chunk;
        rec->help_chunks = nchunks;
        rec->help_on.store(1, std::memory_order_release);
        host_notify(&rec->launched);
        plan_help(rec);
        while (rec->help_done.load(std::memory_order_acquire) < nchunks) std::this_thread::yield();
    } else {
        for (size_t c = 0; c < nchunks; ++c) chunk(c);
    }
    for (size_t c = 0; c < nchunks; ++c) {
        total_tiles += z.part[2 * c];
        *bytes += z.part[2 * c + 1];
    }
    std::memset(&a, 0, sizeof(a));
    a.tile = tile;
    z.starts.clear();
    if (npairs == 0) return MPIXS_SUCCESS;
    const uint64_t nwg = std::min<uint64_t>(total_tiles, uint64_t(w->cfg.batch_max_wg));
    const uint64_t base = total_tiles / nwg;
    const uint64_t extra = total_tiles % nwg;
    if (!SB) {
        z.starts.resize(size_t(nwg));
        SB = z.starts.data();
    }
    uint32_t m = 0;
    uint64_t first_of_m = 0;   // global index of message m's first tile
    for (uint64_t b = 0; b < nwg; ++b) {
        const uint64_t t = b * base + std::min(b, extra);
        while (first_of_m + D[m].ntiles <= t) {
            first_of_m += D[m].ntiles;
            ++m;
        }
        SB[b].msg = m;
        SB[b].tile = uint32_t(t - first_of_m);
    }
    z.nstarts = size_t(nwg);
    a.nmsg = uint32_t(npairs);
    a.desc = D;
    a.start = SB;
    a.base = base;
    a.extra = uint32_t(extra);
    a.tile = tile;
    const int ntc = w->cfg.batch_nontemporal;
    a.nt = (ntc == 1 || (ntc == 0 && *bytes >= (uint64_t(64) << 20))) ? 1u : 0u;
    return MPIXS_SUCCESS;
}

// Last rank of a group: plan it and enqueue wait(all arrivals) + batch
// kernel + signal on its own stream.  Descriptors go to the host-pinned ring
// arena, whose range the signal kernel hands back through a host flag.
int group_launch(World *w, CommShared *sh, GroupRec *rec, int me, StreamObj *st, uint64_t g) {
    const int n = sh->size;
    std::lock_guard<std::mutex> plan_lock(sh->plan_mu);
    BatchArgs a{};
    uint64_t bytes = 0;
    // producer first: the other ranks enqueue their arrival kernels outside
    // the group lock, and the wait for them is enqueued only once all are.
    // Waiting before planning measured faster on large groups (the posting
    // threads slow a concurrent plan) and as fast on small ones.
    int rc = host_wait(w, &rec->posted, [&] { return rec->posted.load(std::memory_order_acquire) >= n - 1; });
    if (rc) return rc;
    // arena range: batch descriptors, workgroup starts (room for as many as a
    // plan may have), merged-reduce descriptors and pointer table, each
    // 256-byte aligned; the plan writes descriptors and starts in place
    const MultiRedPlan &mr = sh->plan.mred;
    int flag = -1;
    uint8_t *h = nullptr;
    size_t bbytes = 0, mdbytes = 0, mpbytes = 0;
    auto reserve = [&](size_t front) -> int {
        bbytes = front;
        mdbytes = mr.on ? (mr.desc.size() * sizeof(MultiRedDesc) + 255) & ~size_t(255) : 0;
        mpbytes = mr.on ? mr.ptrs.size() * sizeof(void *) : 0;
        size_t off = 0;
        const int r = arena_alloc(w, bbytes + mdbytes + mpbytes, &off, &flag);
        if (!r) h = reinterpret_cast<uint8_t *>(w->h_arena + off);
        return r;
    };
    const PlanPlace place = [&](size_t npairs, size_t max_starts, BatchDesc **d, BatchStart **s) -> int {
        const size_t dal = (npairs * sizeof(BatchDesc) + 255) & ~size_t(255);
        const int r = reserve(dal + ((max_starts * sizeof(BatchStart) + 255) & ~size_t(255)));
        if (r) return r;
        *d = reinterpret_cast<BatchDesc *>(h);
        *s = reinterpret_cast<BatchStart *>(h + dal);
        return MPIXS_SUCCESS;
    };
    rc = plan_group(w, sh, rec, n, st, a, &bytes, &place);
    if (rc) return rc;   // the plan fails only before it places anything
    if (!h && mr.on) {
        rc = reserve(0);
        if (rc) return rc;
    }
    // A failed launch before anything that reads the arena range was
    // enqueued hands the range back at once (the ring frees in order, so a
    // range held forever would stall every later group).  After a kernel that
    // reads it was enqueued, the range must stay until that kernel is done:
    // the instance is broken on every rank, so the world is aborted and all
    // of its waits end.
    bool range_read = false;
    auto fail = [&](int code) {
        if (flag >= 0 && !range_read) __atomic_store_n(&w->h_flags[flag], 1u, __ATOMIC_RELEASE);
        if (range_read) mpixs_world_abort(reinterpret_cast<mpixs_world>(w));
        return code;
    };
    uint64_t *arrive = sh->d_grp;
    uint64_t *done = sh->d_grp + 16 * n;
    if (n > 1) {
        WaitArgs wa;
        std::memset(&wa, 0, sizeof(wa));
        for (int q = 0; q < n; ++q) {
            if (q == me) continue;
            wa.ptr[wa.n] = arrive + 16 * q;
            wa.target[wa.n] = g + 1;
            wa.n++;
        }
        rc = do_wait(w, st, wa, MPIXS_TRACE_MATCH);
        if (rc) return fail(rc);
    }
    const size_t nwg = sh->plan.nstarts;
    if (nwg > 0) {
        a.me = st->dev;
        hipEvent_t e0 = nullptr;
        if (profile_on(w)) prof_begin(w, st->hs, &e0);
        rc = gpu_err(launch_batch(st->hs, a, int(nwg)));
        if (profile_on(w)) prof_end(w, st->hs, e0, 0);
        if (rc) return fail(rc);
        range_read = true;
        w->n_copy.fetch_add(1, std::memory_order_relaxed);
        w->bytes_copied.fetch_add(bytes, std::memory_order_relaxed);
    }
    // the group's allreduces, in order (or merged), after its messages
    MultiRedArgs ma{};
    if (mr.on) {
        MultiRedDesc *md = reinterpret_cast<MultiRedDesc *>(h + bbytes);
        const void **mp = reinterpret_cast<const void **>(h + bbytes + mdbytes);
        std::memcpy(md, mr.desc.data(), mr.desc.size() * sizeof(MultiRedDesc));
        std::memcpy(mp, mr.ptrs.data(), mpbytes);
        ma.desc = md;
        ma.ptrs = mp;
        ma.ninst = mr.ninst;
        ma.me = st->dev;
    }
    rc = launch_reds(w, st->hs, sh->plan.reds, mr, ma);
    if (rc) return fail(rc);
    SignalArgs sg;
    std::memset(&sg, 0, sizeof(sg));
    sg.done_ptr = done;
    sg.done_val = g + 1;
    sg.me = st->dev;
    sg.trace = trace_kind(w, 1);
    sg.host_flag = flag >= 0 ? &w->h_flags[flag] : nullptr;
    rc = gpu_err(launch_signal(st->hs, sg));
    if (rc) return fail(rc);
    w->n_post.fetch_add(1, std::memory_order_relaxed);
    return rc;
}

// Last rank of a persistent group: plan it once into device memory, with
// its own relative counters (arrive[q] at word 16q, done at word 16n), and
// optionally build the launching rank's part of a run as a graph.
int batch_create(World *w, CommShared *sh, GroupRec *rec, int me, StreamObj *st,
                 BatchPlan **out, bool static_mem) {
    const int n = sh->size;
    std::unique_ptr<BatchPlan> P(new BatchPlan());
    P->w = w;
    P->n = n;
    P->leader = me;
    P->posted.reset(new std::atomic<uint64_t>[size_t(n)]);
    for (int q = 0; q < n; ++q) P->posted[q].store(0);
    std::lock_guard<std::mutex> plan_lock(sh->plan_mu);
    const std::vector<BatchDesc> &descs = sh->plan.descs;
    const std::vector<BatchStart> &starts = sh->plan.starts;
    int rc = plan_group(w, sh, rec, n, st, P->args, &P->bytes);
    if (rc) return rc;
    P->reds = sh->plan.reds;
    P->mred = sh->plan.mred;
    P->nmsg = descs.size();
    // a group without messages launches no batch kernel in its runs (the
    // graph of an entirely empty group keeps a one-workgroup node)
    P->nwg = std::max(1, int(starts.size()));
    // counters: arrive[q] at word 16q, done at 16n
    const size_t cbytes = size_t(n + 1) * 16 * sizeof(uint64_t);
    const size_t dbytes = (descs.size() * sizeof(BatchDesc) + 255) & ~size_t(255);
    const size_t sbytes = starts.size() * sizeof(BatchStart);
    // merged-reduce descriptors and pointer table after the starts
    const size_t moff = cbytes + dbytes + ((sbytes + 255) & ~size_t(255));
    const size_t mdbytes = P->mred.on ? (P->mred.desc.size() * sizeof(MultiRedDesc) + 255) & ~size_t(255) : 0;
    const size_t mpbytes = P->mred.on ? P->mred.ptrs.size() * sizeof(void *) : 0;
    const size_t total = P->mred.on ? moff + mdbytes + mpbytes : cbytes + dbytes + sbytes;
    if (static_mem) {
        // the device's static region: no allocation; the counters start at
        // zero with the image below
        P->static_mem = true;
        P->device = w->device;
        rc = static_batch_region(w->device, total, &P->d_mem, &P->static_gen);
        if (rc) return rc;
    } else if (hipMalloc(reinterpret_cast<void **>(&P->d_mem), total) != hipSuccess) {
        return MPIXS_ERR_NOMEM;
    }
    std::vector<uint8_t> img(total, 0);
    if (!descs.empty()) std::memcpy(img.data() + cbytes, descs.data(), descs.size() * sizeof(BatchDesc));
    if (!starts.empty()) std::memcpy(img.data() + cbytes + dbytes, starts.data(), sbytes);
    if (P->mred.on) {
        std::memcpy(img.data() + moff, P->mred.desc.data(), P->mred.desc.size() * sizeof(MultiRedDesc));
        std::memcpy(img.data() + moff + mdbytes, P->mred.ptrs.data(), mpbytes);
        P->margs.desc = reinterpret_cast<const MultiRedDesc *>(P->d_mem + moff);
        P->margs.ptrs = reinterpret_cast<const void *const *>(P->d_mem + moff + mdbytes);
        P->margs.ninst = P->mred.ninst;
        P->margs.me = st->dev;
    }
    if (hipMemcpy(P->d_mem, img.data(), img.size(), hipMemcpyHostToDevice) != hipSuccess)
        return MPIXS_ERR_GPU;
    P->d_ctr = reinterpret_cast<uint64_t *>(P->d_mem);
    P->args.desc = reinterpret_cast<const BatchDesc *>(P->d_mem + cbytes);
    P->args.start = reinterpret_cast<const BatchStart *>(P->d_mem + cbytes + dbytes);
    P->args.me = st->dev;
    std::memset(&P->lwait, 0, sizeof(P->lwait));
    P->lwait.ptr0 = P->d_ctr;
    P->lwait.stride = 16;
    P->lwait.n = uint32_t(n);
    P->lwait.skip = uint64_t(1) << me;
    P->lwait.base = P->d_ctr + 16 * n;
    P->lwait.delta = 1;
    P->lwait.ctl = ctl_of(w);
    P->lwait.me = st->dev;
    P->lwait.trace = trace_kind(w, MPIXS_TRACE_MATCH);
    // done + 1 after the batch kernel: the kernel boundary makes its stores
    // visible, so one release store publishes the run (a release in every
    // workgroup instead costs an L2 writeback each and was measured several
    // times slower)
    std::memset(&P->sig, 0, sizeof(P->sig));
    P->sig.done_ptr = P->d_ctr + 16 * n;
    P->sig.inc = 1;
    P->sig.me = st->dev;
    P->sig.trace = trace_kind(w, 1);
    if (w->cfg.batch_sync == 1 && !static_mem) {
        // event dependencies instead of counters: rank q records post_ev[q]
        // after its prior work, the leader's stream waits for those, runs the
        // batch kernel and records done_ev, every other stream waits for it
        P->post_ev.assign(size_t(n), nullptr);
        for (int q = 0; q < n; ++q)
            if (q != me && hipEventCreateWithFlags(&P->post_ev[size_t(q)], hipEventDisableTiming) !=
                               hipSuccess)
                return MPIXS_ERR_GPU;
        if (hipEventCreateWithFlags(&P->done_ev, hipEventDisableTiming) != hipSuccess)
            return MPIXS_ERR_GPU;
    }
    if (w->cfg.batch_graph && !static_mem) {
        hipError_t e = hipSuccess;
        if (P->reds.empty()) {
            e = build_batch_graph(&P->graph, n > 1 ? &P->lwait : nullptr, P->args, P->nwg, P->sig);
        } else {
            // with reductions, record the run by capturing a private stream
            hipStream_t cs = nullptr;
            e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                int r = MPIXS_SUCCESS;
                if (n > 1) r = gpu_err(launch_wait_rel(cs, P->lwait));
                if (!r && P->nmsg > 0) r = gpu_err(launch_batch(cs, P->args, P->nwg));
                if (!r) r = launch_reds(nullptr, cs, P->reds, P->mred, P->margs);
                if (!r) r = gpu_err(launch_signal(cs, P->sig));
                hipGraph_t gr = nullptr;
                const hipError_t e2 = hipStreamEndCapture(cs, &gr);
                P->graph = gr;
                e = r ? hipErrorUnknown : e2;
            }
            if (cs) (void)hipStreamDestroy(cs);
        }
        if (e != hipSuccess || !P->graph ||
            hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0) != hipSuccess)
            return MPIXS_ERR_GPU;
    }
    P->refs.store(n);
    *out = P.release();
    return MPIXS_SUCCESS;
}

int parse_hex(const std::string &s, void *out, size_t n) {
    if (s.size() != 2 * n) return MPIXS_ERR_ARG;
    unsigned char *o = static_cast<unsigned char *>(out);
    for (size_t i = 0; i < n; ++i) {
        unsigned v = 0;
        for (int j = 0; j < 2; ++j) {
            const char ch = s[2 * i + j];
            unsigned d;
            if (ch >= '0' && ch <= '9') d = unsigned(ch - '0');
            else if (ch >= 'a' && ch <= 'f') d = unsigned(ch - 'a' + 10);
            else if (ch >= 'A' && ch <= 'F') d = unsigned(ch - 'A' + 10);
            else return MPIXS_ERR_ARG;
            v = v * 16 + d;
        }
        o[i] = static_cast<unsigned char>(v);
    }
    return MPIXS_SUCCESS;
}

}  // namespace

// ------------------------------------------------------------ Channel
Channel::~Channel() {
    for (Rec *r : recs) delete r;
}

Rec *Channel::at(uint64_t k) {
    while (base + recs.size() <= k) recs.push_back(new Rec());
    return recs[k - base];
}

void Channel::collect() {
    while (!recs.empty() && recs.front()->refs.load(std::memory_order_acquire) == 0) {
        delete recs.front();
        recs.pop_front();
        ++base;
    }
}

CommShared::~CommShared() {
    if (w && !dir.empty()) {
        // every message of the communicator has been waited for: a channel's
        // block frees once its last wait has passed (blocks of channels that
        // never became quiescent stay with the pool)
        std::lock_guard<std::mutex> g(w->chan_mu);
        auto &dr = w->chan_drain;
        dr.erase(std::remove_if(dr.begin(), dr.end(), [&](Channel *ch) { return ch->owner == this; }),
                 dr.end());
        for (auto &kv : dir) {
            Channel *ch = kv.second;
            if (ch->idx != kNoBlock && ch->drain_val && ch->seq[0] == ch->drain_seq &&
                ch->seq[1] == ch->drain_seq)
                w->chan_limbo.emplace_back(ch->idx, ch->drain_val);
        }
    }
    for (auto &kv : dir) delete kv.second;
    for (CollRec *r : colls) delete r;
    for (CollRec *r : hcolls) delete r;
    for (GroupRec *r : groups) delete r;
}

BatchPlan::~BatchPlan() {
    for (hipEvent_t e : post_ev)
        if (e) (void)hipEventDestroy(e);
    if (done_ev) (void)hipEventDestroy(done_ev);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (d_mem && !static_mem) (void)hipFree(d_mem);
}

}  // namespace mpixs

using namespace mpixs;

extern "C" {

// ================================================================== world
int mpixs_world_create(int nranks, const mpixs_config *cfg, mpixs_world *out) {
    if (!out || nranks < 1 || nranks > 4096) return MPIXS_ERR_ARG;
    World *w = new World();
    w->nranks = nranks;
    if (cfg) w->cfg = *cfg;
    mpixs_config &c = w->cfg;
    if (c.max_streams <= 0) c.max_streams = 256;
    // fused (at most 32 workgroups, wait inside) up to 64 KiB: above it a
    // full-grid copy between a wait and a signal kernel is faster despite
    // the two extra launches (ring-halo sweep of the plain enqueue path)
    if (c.fuse_max_bytes == 0) c.fuse_max_bytes = 64 << 10;
    if (c.timeout_ms <= 0) c.timeout_ms = 30000;
    if (c.max_channels <= 0) c.max_channels = 1 << 20;
    if (c.max_collectives <= 0) c.max_collectives = 4096;
    if (c.batch_tile == 0) c.batch_tile = int32_t(BATCH_TILE_DEFAULT);
    // two tiles per workgroup on the 10,000-message batch (a sweep of 8192
    // .. 65536 put 32768 first, 6 % ahead of 16384)
    if (c.batch_max_wg <= 0) c.batch_max_wg = 32768;
    if (c.eager_max_bytes == 0) c.eager_max_bytes = 64 << 10;
    if (c.eager_arena_mib <= 0) c.eager_arena_mib = 64;
    if (!batch_tile_ok(uint32_t(c.batch_tile)) || c.batch_max_wg > (1 << 20) ||
        c.batch_graph < 0 || c.batch_graph > 1 || c.batch_nontemporal < 0 ||
        c.batch_nontemporal > 2 || c.matching < 0 || c.matching > 1 || c.batch_sync < 0 ||
        c.batch_sync > 1 || (c.batch_sync == 1 && c.batch_graph == 1) || c.eager_max_bytes < -1 ||
        c.eager_arena_mib > 65536 || c.trace_events < 0 || c.trace_events > (1 << 24)) {
        delete w;
        return MPIXS_ERR_ARG;
    }
    if (hipGetDevice(&w->device) != hipSuccess) {
        delete w;
        return MPIXS_ERR_GPU;
    }
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, w->device) != hipSuccess ||
        rate_khz <= 0)
        rate_khz = 100000;
    w->timeout_ticks = uint64_t(c.timeout_ms) * uint64_t(rate_khz);
    w->trace_rate_khz = rate_khz;
    static_batch_setup(w->device);

    w->stream_cap = std::max(1024, 4 * c.max_streams);
    w->chan_cap = uint32_t(c.max_channels);
    w->coll_words = size_t(c.max_collectives) * 16;
    const size_t s_bytes = size_t(w->stream_cap) * sizeof(DevStream);
    const size_t c_bytes = size_t(w->chan_cap) * sizeof(DevChan);
    const size_t k_bytes = w->coll_words * sizeof(uint64_t);
    const size_t total = s_bytes + c_bytes + k_bytes;
    if (hipMalloc(reinterpret_cast<void **>(&w->d_pool), total) != hipSuccess) {
        delete w;
        return MPIXS_ERR_NOMEM;
    }
    if (hipMemset(w->d_pool, 0, total) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(w->d_pool);
        delete w;
        return MPIXS_ERR_GPU;
    }
    w->stage.bytes = size_t(c.eager_arena_mib) << 20;
    w->stage.nflags = 16384;
    if (c.eager_max_bytes > 0 &&
        hipMalloc(reinterpret_cast<void **>(&w->stage.base), w->stage.bytes) != hipSuccess) {
        (void)hipFree(w->d_pool);
        delete w;
        return MPIXS_ERR_NOMEM;
    }
    w->d_streams = reinterpret_cast<DevStream *>(w->d_pool);
    if (c.trace_events > 0) {
        // the ring, and every stream block pointing at it (blocks are only
        // ever handed out from this pool, so this is done once)
        w->trace_cap = 1;
        while (w->trace_cap < uint64_t(c.trace_events)) w->trace_cap <<= 1;
        std::vector<DevStream> blocks(static_cast<size_t>(w->stream_cap));
        bool ok = hipMalloc(reinterpret_cast<void **>(&w->d_trace), w->trace_cap * sizeof(TraceEv)) ==
                      hipSuccess &&
                  hipMalloc(reinterpret_cast<void **>(&w->d_trace_head), sizeof(uint64_t)) ==
                      hipSuccess &&
                  hipMemset(w->d_trace_head, 0, sizeof(uint64_t)) == hipSuccess;
        for (size_t i = 0; ok && i < blocks.size(); ++i) {
            std::memset(&blocks[i], 0, sizeof(DevStream));
            blocks[i].trace = w->d_trace;
            blocks[i].trace_head = w->d_trace_head;
            blocks[i].trace_mask = uint32_t(w->trace_cap - 1);
            blocks[i].slot = uint32_t(i);
        }
        ok = ok && hipMemcpy(w->d_streams, blocks.data(), blocks.size() * sizeof(DevStream),
                             hipMemcpyHostToDevice) == hipSuccess;
        if (!ok) {
            if (w->d_trace) (void)hipFree(w->d_trace);
            if (w->d_trace_head) (void)hipFree(w->d_trace_head);
            if (w->stage.base) (void)hipFree(w->stage.base);
            (void)hipFree(w->d_pool);
            delete w;
            return MPIXS_ERR_NOMEM;
        }
    }
    w->d_chans = reinterpret_cast<DevChan *>(w->d_pool + s_bytes);
    w->d_coll = reinterpret_cast<uint64_t *>(w->d_pool + s_bytes + c_bytes);
    if (c.batch_arena_mib <= 0) c.batch_arena_mib = 64;
    w->arena_bytes = size_t(c.batch_arena_mib) << 20;
    w->nflags = 4096;
    // coherent host memory: the host writes these (or reads what the GPU
    // wrote) while kernels run, and kernels must never see a cached copy
    if (hipHostMalloc(reinterpret_cast<void **>(&w->h_abort), 64, hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&w->h_arena), w->arena_bytes,
                      hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&w->h_flags), sizeof(uint32_t) * size_t(w->nflags),
                      hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&w->h_rel), sizeof(uint64_t) * size_t(w->chan_cap),
                      hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&w->stage.flags),
                      sizeof(uint32_t) * size_t(w->stage.nflags), hipHostMallocCoherent) != hipSuccess) {
        (void)hipFree(w->d_pool);
        if (w->stage.base) (void)hipFree(w->stage.base);
        if (w->d_trace) (void)hipFree(w->d_trace);
        if (w->d_trace_head) (void)hipFree(w->d_trace_head);
        if (w->h_abort) (void)hipHostFree(w->h_abort);
        if (w->h_arena) (void)hipHostFree(w->h_arena);
        if (w->h_flags) (void)hipHostFree(w->h_flags);
        if (w->h_rel) (void)hipHostFree(w->h_rel);
        delete w;
        return MPIXS_ERR_NOMEM;
    }
    std::memset(w->h_rel, 0, sizeof(uint64_t) * size_t(w->chan_cap));
    *w->h_abort = 0;
    std::memset(w->h_flags, 0, sizeof(uint32_t) * size_t(w->nflags));
    for (int i = w->nflags - 1; i >= 0; --i) w->free_flags.push_back(i);
    std::memset(w->stage.flags, 0, sizeof(uint32_t) * size_t(w->stage.nflags));
    for (int i = w->stage.nflags - 1; i >= 0; --i) w->stage.free_flags.push_back(i);
    w->ep_users.assign(size_t(c.max_streams), 0);

    CommShared *sh = new CommShared();
    sh->w = w;
    sh->size = nranks;
    sh->id = 0;
    sh->streams.assign(size_t(nranks), nullptr);
    sh->mq.reset(new MatchQueue[size_t(nranks)]);
    sh->handles.store(nranks);
    w->world_sh = sh;
    for (int r = 0; r < nranks; ++r) {
        mpixs_comm_s *h = new mpixs_comm_s();
        h->sh = sh;
        h->rank = r;
        h->world_handle = true;
        w->world_handles.push_back(h);
    }
    *out = static_cast<mpixs_world>(w);
    return MPIXS_SUCCESS;
}

int mpixs_world_comm(mpixs_world w, int rank, mpixs_comm *comm) {
    if (!w || !comm || rank < 0 || rank >= w->nranks) return MPIXS_ERR_ARG;
    *comm = w->world_handles[size_t(rank)];
    return MPIXS_SUCCESS;
}

int mpixs_world_free(mpixs_world *pw) {
    if (!pw || !*pw) return MPIXS_ERR_ARG;
    World *w = *pw;
    {
        std::lock_guard<std::mutex> g(w->reg_mu);
        if (!w->streams.empty() || w->live_comms.load() > 0) return MPIXS_ERR_PENDING;
    }
    {
        std::lock_guard<std::mutex> g(w->prof_mu);
        for (auto &p : w->prof) {
            (void)hipEventDestroy(p.e0);
            (void)hipEventDestroy(p.e1);
        }
        w->prof.clear();
    }
    (void)hipDeviceSynchronize();
    (void)hipFree(w->d_pool);
    (void)hipHostFree(w->h_abort);
    (void)hipHostFree(w->h_arena);
    (void)hipHostFree(w->h_flags);
    (void)hipHostFree(w->h_rel);
    if (w->stage.base) (void)hipFree(w->stage.base);
    (void)hipHostFree(w->stage.flags);
    if (w->d_trace) (void)hipFree(w->d_trace);
    if (w->d_trace_head) (void)hipFree(w->d_trace_head);
    for (auto *h : w->world_handles) delete h;
    delete w->world_sh;
    delete w;
    *pw = nullptr;
    return MPIXS_SUCCESS;
}

int mpixs_world_wait(mpixs_world w, int timeout_ms) {
    if (!w) return MPIXS_ERR_ARG;
    std::vector<hipStream_t> hs;
    {
        std::lock_guard<std::mutex> g(w->reg_mu);
        for (auto *s : w->streams)
            if (s->gpu) hs.push_back(s->hs);
    }
    const auto t0 = std::chrono::steady_clock::now();
    for (hipStream_t s : hs) {
        for (;;) {
            hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) break;
            if (e == hipErrorNotReady) (void)hipGetLastError();
            if (e != hipErrorNotReady) return MPIXS_ERR_GPU;
            if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(timeout_ms))
                return MPIXS_ERR_TIMEOUT;
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
    }
    return MPIXS_SUCCESS;
}

int mpixs_world_abort(mpixs_world w) {
    if (!w) return MPIXS_ERR_ARG;
    w->aborted.store(1, std::memory_order_release);
    __atomic_store_n(w->h_abort, 1u, __ATOMIC_RELEASE);
    host_notify_all();
    return MPIXS_SUCCESS;
}

// =================================================================== info
int mpixs_info_create(mpixs_info *info) {
    if (!info) return MPIXS_ERR_ARG;
    *info = new mpixs_info_s();
    return MPIXS_SUCCESS;
}

int mpixs_info_set(mpixs_info info, const char *key, const char *value) {
    if (!info || !key || !value) return MPIXS_ERR_ARG;
    info->kv[key] = value;
    return MPIXS_SUCCESS;
}

int mpixs_info_set_hex(mpixs_info info, const char *key, const void *value, int vallen) {
    if (!info || !key || (vallen > 0 && !value) || vallen < 0) return MPIXS_ERR_ARG;
    static const char digits[] = "0123456789abcdef";
    std::string s;
    s.reserve(size_t(vallen) * 2);
    const unsigned char *p = static_cast<const unsigned char *>(value);
    for (int i = 0; i < vallen; ++i) {
        s.push_back(digits[p[i] >> 4]);
        s.push_back(digits[p[i] & 15]);
    }
    info->kv[key] = s;
    return MPIXS_SUCCESS;
}

int mpixs_info_get(mpixs_info info, const char *key, char *value, int valuelen, int *flag) {
    if (!info || !key || !flag) return MPIXS_ERR_ARG;
    auto it = info->kv.find(key);
    *flag = it != info->kv.end();
    if (*flag && value && valuelen > 0) {
        std::snprintf(value, size_t(valuelen), "%s", it->second.c_str());
    }
    return MPIXS_SUCCESS;
}

int mpixs_info_free(mpixs_info *info) {
    if (!info || !*info) return MPIXS_ERR_ARG;
    delete *info;
    *info = nullptr;
    return MPIXS_SUCCESS;
}

// ================================================================= stream
int mpixs_stream_create(mpixs_world w, mpixs_info info, mpixs_stream *out) {
    if (!w || !out) return MPIXS_ERR_ARG;
    bool gpu = false;
    hipStream_t hs = nullptr;
    if (info) {
        auto t = info->kv.find("type");
        if (t != info->kv.end()) {
            if (t->second != "hipStream_t") return MPIXS_ERR_ARG;
            auto v = info->kv.find("value");
            if (v == info->kv.end()) return MPIXS_ERR_ARG;
            if (parse_hex(v->second, &hs, sizeof(hs))) return MPIXS_ERR_ARG;
            gpu = true;
        }
    }
    int ep = -1;
    {
        std::lock_guard<std::mutex> g(w->ep_mu);
        for (int i = 0; i < w->cfg.max_streams; ++i)
            if (w->ep_users[size_t(i)] == 0) {
                ep = i;
                break;
            }
        if (ep < 0) {
            if (w->cfg.endpoint_policy != 1) return MPIXS_ERR_NO_ENDPOINT;
            ep = w->ep_rr;
            w->ep_rr = (w->ep_rr + 1) % w->cfg.max_streams;
        }
        // a block a freed stream returned (clean: no error recorded), else a
        // fresh one; a returned block keeps its ticket count, which the new
        // stream continues from
        int slot;
        uint64_t tickets = 0;
        if (!w->stream_free.empty()) {
            slot = w->stream_free.back().first;
            tickets = w->stream_free.back().second;
            w->stream_free.pop_back();
            w->streams_recycled.fetch_add(1, std::memory_order_relaxed);
        } else {
            slot = w->stream_next.fetch_add(1);
            if (slot >= w->stream_cap) return MPIXS_ERR_NOMEM;
        }
        w->ep_users[size_t(ep)]++;
        mpixs_stream_s *s = new mpixs_stream_s();
        s->w = w;
        s->gpu = gpu;
        s->hs = hs;
        s->endpoint = ep;
        s->dev = w->d_streams + slot;
        s->tickets = tickets;
        s->id = w->next_stream_id.fetch_add(1);
        *out = s;
    }
    {
        std::lock_guard<std::mutex> g(w->reg_mu);
        w->streams.insert(*out);
    }
    return MPIXS_SUCCESS;
}

int mpixs_stream_free(mpixs_stream *ps) {
    if (!ps || !*ps) return MPIXS_ERR_ARG;
    mpixs_stream_s *s = *ps;
    World *w = s->w;
    if (s->comm_refs.load() > 0) return MPIXS_ERR_PENDING;
    if (s->gpu) {
        hipError_t e = hipStreamQuery(s->hs);
        if (e == hipErrorNotReady) {
            (void)hipGetLastError();   // not an error of a later call
            return MPIXS_ERR_PENDING;
        }
    }
    // The stream is idle, and every kernel of another stream that writes its
    // block (a batch recording a receive's error) was waited for on it: the
    // block may go to the next stream if it holds no error (a read on the
    // idle stream itself); a block with an error stays out of use.
    bool clean = true;
    if (s->gpu) {
        uint32_t v[2] = {1, 1};
        clean = hipMemcpyAsync(v, &s->dev->first_error, sizeof(v), hipMemcpyDeviceToHost,
                               s->hs) == hipSuccess &&
                hipStreamSynchronize(s->hs) == hipSuccess && v[0] == 0 && v[1] == 0;
    }
    {
        std::lock_guard<std::mutex> g(w->ep_mu);
        w->ep_users[size_t(s->endpoint)]--;
        if (clean) w->stream_free.emplace_back(int(s->dev - w->d_streams), s->tickets);
    }
    {
        std::lock_guard<std::mutex> g(w->reg_mu);
        w->streams.erase(s);
    }
    delete s;
    *ps = nullptr;
    return MPIXS_SUCCESS;
}

int mpixs_stream_get_error(mpixs_stream s, int *first_error) {
    if (!s || !first_error) return MPIXS_ERR_ARG;
    uint32_t v = 0;
    // read on the stream itself, so no other stream is waited for
    if (!s->gpu) {
        *first_error = 0;
        return MPIXS_SUCCESS;
    }
    if (hipMemcpyAsync(&v, &s->dev->first_error, sizeof(v), hipMemcpyDeviceToHost, s->hs) !=
            hipSuccess ||
        hipStreamSynchronize(s->hs) != hipSuccess)
        return MPIXS_ERR_GPU;
    *first_error = int(v);
    return MPIXS_SUCCESS;
}

// ========================================================== communicator
namespace {

// Collective lines for a new communicator: the lines of a freed one of the
// same size once no stream its ranks used can still run one of its kernels
// (each is freed, or idle now), else fresh lines, else (pool exhausted) the
// first freed lines of that size after synchronising their live streams.
// Floors: the instance numbers to start from.
int take_coll_lines(World *w, size_t words, size_t *off, uint64_t *floor_coll,
                    uint64_t *floor_group) {
    std::lock_guard<std::mutex> g(w->coll_mu);
    // users still alive (same object and id), under the registry lock
    auto live_users = [&](const CollLines &cl) {
        std::vector<hipStream_t> hs;
        std::lock_guard<std::mutex> g2(w->reg_mu);
        for (const auto &u : cl.users) {
            auto it = w->streams.find(u.first);
            if (it != w->streams.end() && (*it)->id == u.second && (*it)->gpu)
                hs.push_back((*it)->hs);
        }
        return hs;
    };
    auto take = [&](size_t i) {
        const CollLines &cl = w->coll_free[i];
        *off = cl.off;
        *floor_coll = cl.floor_coll;
        *floor_group = cl.floor_group;
        w->coll_free.erase(w->coll_free.begin() + long(i));
        w->colls_recycled.fetch_add(1, std::memory_order_relaxed);
        return MPIXS_SUCCESS;
    };
    for (size_t i = 0; i < w->coll_free.size(); ++i) {
        if (w->coll_free[i].words != words) continue;
        bool idle = true;
        for (hipStream_t h : live_users(w->coll_free[i])) {
            const hipError_t q = hipStreamQuery(h);
            if (q == hipErrorNotReady) (void)hipGetLastError();
            if (q != hipSuccess) {
                idle = false;
                break;
            }
        }
        if (idle) return take(i);
    }
    if (w->coll_next.load() + words <= w->coll_words) {
        const size_t o = w->coll_next.fetch_add(words);
        if (o + words <= w->coll_words) {
            *off = o;
            *floor_coll = *floor_group = 0;
            return MPIXS_SUCCESS;
        }
    }
    for (size_t i = 0; i < w->coll_free.size(); ++i) {
        if (w->coll_free[i].words != words) continue;
        for (hipStream_t h : live_users(w->coll_free[i]))
            if (hipStreamSynchronize(h) != hipSuccess) return MPIXS_ERR_GPU;
        return take(i);
    }
    return MPIXS_ERR_NOMEM;
}

}  // namespace

int mpixs_comm_create_with_stream(mpixs_comm parent, mpixs_stream s, mpixs_comm *newcomm) {
    if (!parent || !parent->sh || !newcomm) return MPIXS_ERR_COMM;
    CommShared *ps = parent->sh;
    World *w = ps->w;
    if (s && s->w != w) return MPIXS_ERR_STREAM;
    const uint64_t k = parent->create_seq++;
    CommShared *sh = nullptr;
    {
        std::unique_lock<std::mutex> g(ps->create_mu);
        CreateRec &cr = ps->creates[k];
        if (!cr.sh) {
            const size_t words = size_t(16) * size_t(ps->size + 1);
            size_t off = 0;
            uint64_t fc = 0, fg = 0;
            const int rc0 = take_coll_lines(w, 2 * words, &off, &fc, &fg);
            if (rc0) return rc0;
            cr.sh = new CommShared();
            cr.sh->w = w;
            cr.sh->size = ps->size;
            cr.sh->id = w->next_comm_id.fetch_add(1);
            cr.sh->streams.assign(size_t(ps->size), nullptr);
            cr.sh->mq.reset(new MatchQueue[size_t(ps->size)]);
            cr.sh->d_coll = w->d_coll + off;
            cr.sh->d_grp = w->d_coll + off + words;
            cr.sh->coll_off = off;
            cr.sh->coll_words = 2 * words;
            cr.sh->floor_coll = cr.sh->coll_base = cr.sh->max_coll = fc;
            cr.sh->floor_group = cr.sh->group_base = cr.sh->max_group = fg;
        }
        cr.sh->streams[size_t(parent->rank)] = s;
        cr.arrived++;
        sh = cr.sh;
    }
    host_notify(&ps->creates);
    // all ranks of the parent must arrive (a collective call, §3.3)
    int rc = host_wait(w, &ps->creates, [&] {
        std::lock_guard<std::mutex> g(ps->create_mu);
        return ps->creates[k].arrived == ps->size;
    });
    {
        std::lock_guard<std::mutex> g(ps->create_mu);
        CreateRec &cr = ps->creates[k];
        if (++cr.left == ps->size) ps->creates.erase(k);
    }
    if (rc) return rc;
    mpixs_comm_s *c = new mpixs_comm_s();
    c->sh = sh;
    c->rank = parent->rank;
    c->stream = s;
    c->coll_seq = sh->floor_coll;
    c->group_seq = sh->floor_group;
    if (s) s->comm_refs.fetch_add(1);
    sh->handles.fetch_add(1);
    w->live_comms.fetch_add(1);
    *newcomm = c;
    return MPIXS_SUCCESS;
}

int mpixs_comm_free(mpixs_comm *pc) {
    if (!pc || !*pc) return MPIXS_ERR_ARG;
    mpixs_comm_s *c = *pc;
    if (c->world_handle) return MPIXS_ERR_COMM;
    if (c->pending.load() > 0) return MPIXS_ERR_PENDING;
    World *w = c->sh->w;
    CommShared *sh = c->sh;
    if (sh->coll_words) {
        // what this rank leaves for the reuse of the collective lines: its
        // instance counts, and the stream its kernels ran on
        std::lock_guard<std::mutex> g(sh->free_mu);
        sh->max_coll = std::max(sh->max_coll, c->coll_seq);
        sh->max_group = std::max(sh->max_group, c->group_seq);
        if (c->stream) sh->users.emplace_back(c->stream, c->stream->id);
    }
    if (c->stream) c->stream->comm_refs.fetch_sub(1);
    for (StreamObj *s : c->mstreams) s->comm_refs.fetch_sub(1);
    if (sh->handles.fetch_sub(1) == 1) {
        if (sh->coll_words) {
            CollLines cl;
            cl.off = sh->coll_off;
            cl.words = sh->coll_words;
            cl.floor_coll = sh->max_coll;
            cl.floor_group = sh->max_group;
            cl.users.swap(sh->users);
            std::lock_guard<std::mutex> g(w->coll_mu);
            w->coll_free.push_back(std::move(cl));
        }
        delete sh;
    }
    w->live_comms.fetch_sub(1);
    delete c;
    *pc = nullptr;
    return MPIXS_SUCCESS;
}

int mpixs_comm_rank(mpixs_comm c, int *rank) {
    if (!c || !rank) return MPIXS_ERR_ARG;
    *rank = c->rank;
    return MPIXS_SUCCESS;
}

int mpixs_comm_size(mpixs_comm c, int *size) {
    if (!c || !size) return MPIXS_ERR_ARG;
    *size = c->sh->size;
    return MPIXS_SUCCESS;
}

// ================================================================ enqueue
int mpixs_send_enqueue(const void *buf, int count, mpixs_datatype dt, int dest, int tag,
                       mpixs_comm comm) {
    return p2p(comm, 0, buf, count, dt, dest, tag, nullptr, nullptr);
}

int mpixs_recv_enqueue(void *buf, int count, mpixs_datatype dt, int source, int tag,
                       mpixs_comm comm, mpixs_status *status) {
    return p2p(comm, 1, buf, count, dt, source, tag, status, nullptr);
}

int mpixs_isend_enqueue(const void *buf, int count, mpixs_datatype dt, int dest, int tag,
                        mpixs_comm comm, mpixs_request *request) {
    if (!request) return MPIXS_ERR_ARG;
    return p2p(comm, 0, buf, count, dt, dest, tag, nullptr, request);
}

int mpixs_irecv_enqueue(void *buf, int count, mpixs_datatype dt, int source, int tag,
                        mpixs_comm comm, mpixs_request *request) {
    if (!request) return MPIXS_ERR_ARG;
    return p2p(comm, 1, buf, count, dt, source, tag, nullptr, request);
}

// ------------------------------------------- multiplex communicators (§3.5)
}  // extern "C"

namespace {

// Argument checks of the index-addressed calls, in the order of check_p2p
// (communicator, count, datatype, peer, tag, stream indices, overlap, size
// limit, buffer).  The local index names the stream the operation is enqueued on.
int check_mp(mpixs_comm_s *c, const void *buf, int count, mpixs_datatype dt, int peer, int tag,
             bool recv, int src_idx, int dst_idx, const TypeObj **t, StreamObj **st) {
    if (!c || !c->sh || !c->sh->multiplex) return MPIXS_ERR_COMM;
    CommShared *sh = c->sh;
    if (count < 0) return MPIXS_ERR_COUNT;
    if (!type_ok(dt, t)) return MPIXS_ERR_TYPE;
    if (!(recv && peer == MPIXS_ANY_SOURCE) && (peer < 0 || peer >= sh->size)) return MPIXS_ERR_RANK;
    if (!(recv && tag == MPIXS_ANY_TAG) && tag < 0) return MPIXS_ERR_TAG;
    const int local = recv ? dst_idx : src_idx;
    const int remote = recv ? src_idx : dst_idx;
    if (local < 0 || local >= int(c->mstreams.size())) return MPIXS_ERR_RANK;
    if (recv && remote == MPIXS_ANY_INDEX) {
    } else if (recv && peer == MPIXS_ANY_SOURCE) {
        if (remote < 0) return MPIXS_ERR_RANK;
    } else if (remote < 0 || remote >= int(sh->mst[size_t(peer)].size())) {
        return MPIXS_ERR_RANK;
    }
    if (recv && count > 0 && (*t)->L.overlap) return MPIXS_ERR_TYPE;
    const int64_t bytes = int64_t(count) * (*t)->L.size;
    if (!(*t)->L.dense() && bytes >= (int64_t(1) << 32)) return MPIXS_ERR_COUNT;
    if (bytes > 0) {
        int64_t lo, hi;
        type_span(*t, count, &lo, &hi);
        const int rc = check_buf(c->mstreams[size_t(local)], buf, lo, hi, false);
        if (rc) return rc;
    }
    if (sh->w->aborted.load()) return MPIXS_ERR_ABORTED;
    *st = c->mstreams[size_t(local)];
    return MPIXS_SUCCESS;
}

int mp_p2p(mpixs_comm_s *c, int side, const void *buf, int count, mpixs_datatype dt, int peer,
           int tag, int src_idx, int dst_idx, mpixs_status *status, mpixs_request *req) {
    const TypeObj *t = nullptr;
    StreamObj *st = nullptr;
    int rc = check_mp(c, buf, count, dt, peer, tag, side == 1, src_idx, dst_idx, &t, &st);
    if (!rc && status) rc = check_buf(st, status, 0, sizeof(mpixs_status), true);
    if (rc) return rc;
    return side == 0 ? p2p_queue(c, 0, buf, count, t, peer, tag, status, req, st, src_idx, dst_idx)
                     : p2p_queue(c, 1, buf, count, t, peer, tag, status, req, st, dst_idx, src_idx);
}

}  // namespace

extern "C" {

int mpixs_stream_send_enqueue(const void *buf, int count, mpixs_datatype dt, int dest, int tag,
                              mpixs_comm comm, int src_idx, int dst_idx) {
    return mp_p2p(comm, 0, buf, count, dt, dest, tag, src_idx, dst_idx, nullptr, nullptr);
}

int mpixs_stream_recv_enqueue(void *buf, int count, mpixs_datatype dt, int source, int tag,
                              mpixs_comm comm, int src_idx, int dst_idx, mpixs_status *status) {
    return mp_p2p(comm, 1, buf, count, dt, source, tag, src_idx, dst_idx, status, nullptr);
}

int mpixs_stream_isend_enqueue(const void *buf, int count, mpixs_datatype dt, int dest, int tag,
                               mpixs_comm comm, int src_idx, int dst_idx, mpixs_request *request) {
    if (!request) return MPIXS_ERR_ARG;
    return mp_p2p(comm, 0, buf, count, dt, dest, tag, src_idx, dst_idx, nullptr, request);
}

int mpixs_stream_irecv_enqueue(void *buf, int count, mpixs_datatype dt, int source, int tag,
                               mpixs_comm comm, int src_idx, int dst_idx, mpixs_request *request) {
    if (!request) return MPIXS_ERR_ARG;
    return mp_p2p(comm, 1, buf, count, dt, source, tag, src_idx, dst_idx, nullptr, request);
}

int mpixs_comm_create_multiplex(mpixs_comm parent, int count, const mpixs_stream *streams,
                                mpixs_comm *newcomm) {
    if (!parent || !parent->sh || !newcomm) return MPIXS_ERR_COMM;
    if (count < 0 || count > 64 || (count > 0 && !streams)) return MPIXS_ERR_ARG;
    CommShared *ps = parent->sh;
    World *w = ps->w;
    for (int i = 0; i < count; ++i)
        if (!streams[i] || streams[i]->w != w || !streams[i]->gpu) return MPIXS_ERR_STREAM;
    const uint64_t k = parent->create_seq++;
    CommShared *sh = nullptr;
    {
        std::unique_lock<std::mutex> g(ps->create_mu);
        CreateRec &cr = ps->creates[k];
        if (!cr.sh) {
            cr.sh = new CommShared();
            cr.sh->w = w;
            cr.sh->size = ps->size;
            cr.sh->id = w->next_comm_id.fetch_add(1);
            cr.sh->streams.assign(size_t(ps->size), nullptr);
            cr.sh->multiplex = true;
            cr.sh->mst.resize(size_t(ps->size));
        }
        cr.sh->mst[size_t(parent->rank)].assign(streams, streams + count);
        cr.arrived++;
        sh = cr.sh;
    }
    host_notify(&ps->creates);
    // all ranks of the parent must arrive (a collective call, §3.3 / §3.5)
    int rc = host_wait(w, &ps->creates, [&] {
        std::lock_guard<std::mutex> g(ps->create_mu);
        return ps->creates[k].arrived == ps->size;
    });
    {
        std::lock_guard<std::mutex> g(ps->create_mu);
        if (!rc && !sh->ep_ready) {
            // the first rank past the barrier lays out the endpoints
            sh->ep_base.assign(size_t(ps->size) + 1, 0);
            for (int q = 0; q < ps->size; ++q)
                sh->ep_base[size_t(q) + 1] = sh->ep_base[size_t(q)] + int(sh->mst[size_t(q)].size());
            sh->mq.reset(new MatchQueue[size_t(std::max(1, sh->ep_base[size_t(ps->size)]))]);
            sh->ep_ready = true;
        }
        CreateRec &cr = ps->creates[k];
        if (++cr.left == ps->size) ps->creates.erase(k);
    }
    if (rc) return rc;
    mpixs_comm_s *c = new mpixs_comm_s();
    c->sh = sh;
    c->rank = parent->rank;
    c->stream = nullptr;   // the ordinary calls need a single stream: MPIXS_ERR_COMM
    c->mstreams.assign(streams, streams + count);
    for (StreamObj *s : c->mstreams) s->comm_refs.fetch_add(1);
    sh->handles.fetch_add(1);
    w->live_comms.fetch_add(1);
    *newcomm = c;
    return MPIXS_SUCCESS;
}

int mpixs_wait_enqueue(mpixs_request *request, mpixs_status *status) {
    if (!request) return MPIXS_ERR_REQUEST;
    return wait_many(1, request, status, false);
}

int mpixs_waitall_enqueue(int count, mpixs_request requests[], mpixs_status statuses[]) {
    return wait_many(count, requests, statuses, true);
}

int mpixs_allreduce_enqueue(const void *sendbuf, void *recvbuf, int count, mpixs_datatype dt,
                            mpixs_op op, mpixs_comm c) {
    int rc = check_allreduce(c, sendbuf, recvbuf, count, dt, op, true);
    if (rc) return rc;
    if (c->in_group) {
        // recorded; the group's end reduces it after the group's messages
        GOp g;
        g.kind = 2;
        g.red_in = sendbuf == MPIXS_IN_PLACE ? recvbuf : sendbuf;
        g.red_out = recvbuf;
        g.red_count = count;
        g.red_dtype = dt;
        g.red_op = op;
        g.side.st = c->stream;
        g.side.rank = c->rank;
        c->gops.push_back(g);
        return MPIXS_SUCCESS;
    }
    CommShared *sh = c->sh;
    World *w = sh->w;
    StreamObj *st = c->stream;
    const uint64_t k = c->coll_seq++;
    const int n = sh->size;
    const void *in = sendbuf == MPIXS_IN_PLACE ? recvbuf : sendbuf;
    uint64_t *arrive = sh->d_coll;
    uint64_t *done = sh->d_coll + 16 * n;
    sh->coll_mu.lock();
    CollRec *rec = coll_at(sh->colls, sh->coll_base, k, n);
    rec->in[c->rank] = in;
    rec->out[c->rank] = recvbuf;
    if (rec->arrived == 0) {
        rec->count = count;
        rec->dtype = dt;
        rec->op = op;
    }
    rec->arrived++;
    if (rec->arrived == n) {
        sh->coll_mu.unlock();
        // producer first: the other ranks launch their arrival kernels
        // outside the lock; the reduction that waits for them is enqueued
        // once all are
        rc = host_wait(w, &rec->posted, [&] { return rec->posted.load(std::memory_order_acquire) >= n - 1; });
        if (!rc) rc = do_reduce(w, st, rec, n, c->rank, arrive, k + 1, done, k + 1);
        rec->reduce_enq.store(1, std::memory_order_release);
        host_notify(&rec->reduce_enq);
    } else {
        sh->coll_mu.unlock();
        // counted even when the launch failed, so the reducing rank never
        // waits for it; the failure is this rank's error
        rc = do_post(w, st, arrive + 16 * c->rank, k + 1);
        rec->posted.fetch_add(1, std::memory_order_release);
        host_notify(&rec->posted);
        if (!rc) rc = host_wait(w, &rec->reduce_enq, [&] { return rec->reduce_enq.load(std::memory_order_acquire) != 0; });
        if (!rc) {
            WaitArgs a = wait_one(done, k + 1);
            rc = do_wait(w, st, a, MPIXS_TRACE_COMPLETE);
        }
    }
    if (rec->refs.fetch_sub(1) == 1) {
        std::lock_guard<std::mutex> g(sh->coll_mu);
        coll_collect(sh->colls, sh->coll_base);
    }
    return rc;
}

// ================================================================ groups
int mpixs_group_start(mpixs_comm c) {
    if (!c || !c->sh) return MPIXS_ERR_COMM;
    if (!c->stream || !c->stream->gpu) return MPIXS_ERR_COMM;
    if (c->sh->size > 64) return MPIXS_ERR_COMM;
    if (c->in_group) return MPIXS_ERR_ARG;
    c->in_group = true;
    c->gops.clear();
    return MPIXS_SUCCESS;
}

}  // extern "C"

namespace {

// Collective end of the rank's group; kind 1 runs it once, kind 2 makes it a
// persistent batch (returned in *plan).
int group_finish(mpixs_comm c, int kind, BatchPlan **plan) {
    c->in_group = false;
    CommShared *sh = c->sh;
    World *w = sh->w;
    StreamObj *st = c->stream;
    const int n = sh->size;
    const uint64_t g = c->group_seq++;
    bool unwaited = false;
    for (const GOp &op : c->gops) unwaited = unwaited || op.req != nullptr;
    sh->grp_mu.lock();
    while (sh->group_base + sh->groups.size() <= g) {
        GroupRec *r = new GroupRec();
        r->ops.resize(size_t(n));
        r->streams.assign(size_t(n), nullptr);
        r->refs.store(n);
        sh->groups.push_back(r);
    }
    GroupRec *rec = sh->groups[g - sh->group_base];
    rec->ops[size_t(c->rank)] = std::move(c->gops);
    c->gops.clear();
    rec->streams[size_t(c->rank)] = st;
    if (rec->kind == 0) rec->kind = kind;
    else if (rec->kind != kind) rec->mismatch = true;
    if (kind >= 2 && unwaited) rec->bad = true;
    const bool last = ++rec->arrived == n;
    int rc = MPIXS_SUCCESS;
    if (last) {
        sh->grp_mu.unlock();
        if (rec->mismatch || rec->bad) rc = MPIXS_ERR_ARG;
        else if (kind == 1) rc = group_launch(w, sh, rec, c->rank, st, g);
        else rc = batch_create(w, sh, rec, c->rank, st, &rec->batch, kind == 3);
        rec->error = rc;
        rec->launched.store(1, std::memory_order_release);
        host_notify(&rec->launched);
    } else {
        sh->grp_mu.unlock();
        if (kind == 1) {
            // counted even when the launch failed, so the planning rank
            // never waits for it; the failure is this rank's error
            rc = do_post(w, st, sh->d_grp + 16 * c->rank, g + 1);
            rec->posted.fetch_add(1, std::memory_order_release);
            host_notify(&rec->posted);
        }
        // wait for the launch, taking chunks of the plan when the planning
        // rank publishes them
        auto ready = [&] {
            return rec->launched.load(std::memory_order_acquire) != 0 ||
                   (rec->help_on.load(std::memory_order_acquire) != 0 &&
                    rec->help_next.load(std::memory_order_relaxed) < rec->help_chunks);
        };
        while (!rc) {
            rc = host_wait(w, &rec->launched, ready);
            if (rc || rec->launched.load(std::memory_order_acquire) != 0) break;
            plan_help(rec);
        }
        if (!rc) rc = rec->error;
        if (!rc && kind == 1) {
            WaitArgs a = wait_one(sh->d_grp + 16 * n, g + 1);
            rc = do_wait(w, st, a, MPIXS_TRACE_COMPLETE);
        }
    }
    if (!rc && kind >= 2) *plan = rec->batch;
    if (rec->refs.fetch_sub(1) == 1) {
        std::lock_guard<std::mutex> lk(sh->grp_mu);
        while (!sh->groups.empty() && sh->groups.front()->refs.load() == 0) {
            delete sh->groups.front();
            sh->groups.pop_front();
            ++sh->group_base;
        }
    }
    return rc;
}

}  // namespace

extern "C" {

int mpixs_group_end(mpixs_comm c) {
    if (!c || !c->sh) return MPIXS_ERR_COMM;
    if (!c->in_group) return MPIXS_ERR_ARG;
    return group_finish(c, 1, nullptr);
}

int mpixs_group_end_init(mpixs_comm c, mpixs_batch *batch) {
    if (!c || !c->sh) return MPIXS_ERR_COMM;
    if (!c->in_group || !batch) return MPIXS_ERR_ARG;
    *batch = nullptr;
    BatchPlan *P = nullptr;
    const int rc = group_finish(c, 2, &P);
    if (rc) return rc;
    mpixs_batch_s *b = new mpixs_batch_s();
    b->p = P;
    b->comm = c;
    b->rank = c->rank;
    c->pending.fetch_add(1);
    *batch = b;
    return MPIXS_SUCCESS;
}

int mpixs_group_end_init_static(mpixs_comm c, mpixs_batch *batch) {
    if (!c || !c->sh) return MPIXS_ERR_COMM;
    if (!c->in_group || !batch) return MPIXS_ERR_ARG;
    *batch = nullptr;
    BatchPlan *P = nullptr;
    const int rc = group_finish(c, 3, &P);
    if (rc) return rc;
    mpixs_batch_s *b = new mpixs_batch_s();
    b->p = P;
    b->comm = c;
    b->rank = c->rank;
    c->pending.fetch_add(1);
    *batch = b;
    return MPIXS_SUCCESS;
}

int mpixs_batch_start_enqueue(mpixs_batch b) {
    if (!b || !b->p) return MPIXS_ERR_REQUEST;
    mpixs_comm_s *c = b->comm;
    if (c->in_group) return MPIXS_ERR_ARG;
    BatchPlan *P = b->p;
    // a later static plan on this GPU has overwritten this one's region
    if (P->static_mem && !static_batch_current(P->device, P->static_gen)) return MPIXS_ERR_REQUEST;
    World *w = P->w;
    StreamObj *st = c->stream;
    if (w->aborted.load()) return MPIXS_ERR_ABORTED;
    const uint64_t e = b->runs + 1;
    int rc = MPIXS_SUCCESS;
    if (b->rank == P->leader) {
        // producer first: every other rank's arrival for run e is enqueued
        for (int q = 0; q < P->n && !rc; ++q) {
            if (q == P->leader) continue;
            rc = host_wait(w, &P->posted[q], [&] { return P->posted[q].load(std::memory_order_acquire) >= e; });
        }
        if (!rc) {
            if (P->done_ev) {
                // each follower recorded its event for run e before posting
                // e, and records it again only after its wait for this run,
                // which comes after this launch (followers wait for
                // `launched`), so every wait here sees run e's record
                for (int q = 0; q < P->n && !rc; ++q)
                    if (q != P->leader) rc = gpu_err(hipStreamWaitEvent(st->hs, P->post_ev[size_t(q)], 0));
                if (!rc && P->nmsg > 0) rc = gpu_err(launch_batch(st->hs, P->args, P->nwg));
                if (!rc) rc = launch_reds(w, st->hs, P->reds, P->mred, P->margs);
                if (!rc) rc = gpu_err(hipEventRecord(P->done_ev, st->hs));
            } else if (P->exec) {
                rc = gpu_err(hipGraphLaunch(P->exec, st->hs));
                if (!rc) count_reds(w, P->reds, P->mred);
            } else {
                if (P->n > 1) rc = gpu_err(launch_wait_rel(st->hs, P->lwait));
                if (!rc && P->nmsg > 0) rc = gpu_err(launch_batch(st->hs, P->args, P->nwg));
                if (!rc) rc = launch_reds(w, st->hs, P->reds, P->mred, P->margs);
                if (!rc) rc = gpu_err(launch_signal(st->hs, P->sig));
            }
        }
        if (rc) {
            int z = 0;
            P->launch_err.compare_exchange_strong(z, rc);
        }
        P->launched.store(e, std::memory_order_release);
        host_notify(&P->launched);
        if (!rc) {
            w->n_copy.fetch_add(P->nmsg > 0 ? 1 : 0, std::memory_order_relaxed);
            w->bytes_copied.fetch_add(P->bytes, std::memory_order_relaxed);
        }
    } else {
        if (P->done_ev) rc = gpu_err(hipEventRecord(P->post_ev[size_t(b->rank)], st->hs));
        else rc = gpu_err(launch_post_inc(st->hs, P->d_ctr + 16 * b->rank, trace_of(w, st)));
        if (rc) return rc;
        P->posted[b->rank].store(e, std::memory_order_release);
        host_notify(&P->posted[b->rank]);
        w->n_post.fetch_add(1, std::memory_order_relaxed);
        rc = host_wait(w, &P->launched, [&] { return P->launched.load(std::memory_order_acquire) >= e; });
        if (!rc) rc = P->launch_err.load();
        if (!rc && P->done_ev) {
            // the leader recorded run e's completion before publishing e,
            // and records run e + 1 only after this rank posted e + 1
            rc = gpu_err(hipStreamWaitEvent(st->hs, P->done_ev, 0));
            w->n_wait.fetch_add(1, std::memory_order_relaxed);
        } else if (!rc) {
            RelWaitArgs a;
            std::memset(&a, 0, sizeof(a));
            a.ptr0 = P->d_ctr + 16 * P->n;
            a.n = 1;
            a.base = P->d_ctr + 16 * b->rank;
            a.ctl = ctl_of(w);
            a.me = st->dev;
            a.trace = trace_kind(w, MPIXS_TRACE_COMPLETE);
            rc = gpu_err(launch_wait_rel(st->hs, a));
            w->n_wait.fetch_add(1, std::memory_order_relaxed);
        }
    }
    b->runs = e;
    return rc;
}

int mpixs_batch_free(mpixs_batch *batch) {
    if (!batch || !*batch || !(*batch)->p) return MPIXS_ERR_REQUEST;
    mpixs_batch_s *b = *batch;
    BatchPlan *P = b->p;
    b->comm->pending.fetch_sub(1);
    delete b;
    *batch = nullptr;
    if (P->refs.fetch_sub(1) == 1) {
        // no kernel of any run may still read the plan
        (void)hipDeviceSynchronize();
        delete P;
    }
    return MPIXS_SUCCESS;
}

// ========================================================= host-synchronised
int mpixs_send(const void *buf, int count, mpixs_datatype dt, int dest, int tag, mpixs_comm c) {
    const TypeObj *t = nullptr;
    int rc = check_p2p(c, buf, count, dt, dest, tag, false, &t);
    if (rc) return rc;
    if (c->sh->w->cfg.matching == 1) return MPIXS_ERR_COMM;   // sequence channels only
    World *w = c->sh->w;
    StreamObj *st = c->stream;
    if (hipStreamSynchronize(st->hs) != hipSuccess) return MPIXS_ERR_GPU;
    Channel *ch = get_channel(c, c->rank, dest, tag, true);
    if (!ch) return MPIXS_ERR_NOMEM;
    const uint64_t k = ch->seq[0]++;
    Rec *rec;
    {
        std::lock_guard<std::mutex> g(ch->mu);
        rec = ch->at(k);
        rec->s.buf = buf;
        rec->s.count = count;
        rec->s.t = t;
        rec->s.bytes = int64_t(count) * t->L.size;
        rec->s.st = st;
        rec->s.rank = c->rank;
        rec->arrived.fetch_or(ARR_S, std::memory_order_release);
        host_notify(&rec->arrived);
    }
    rc = host_wait(w, &rec->done_host, [&] { return rec->done_host.load(std::memory_order_acquire) != 0; });
    rec_release(ch, rec);
    return rc;
}

int mpixs_recv(void *buf, int count, mpixs_datatype dt, int source, int tag, mpixs_comm c,
               mpixs_status *status) {
    const TypeObj *t = nullptr;
    int rc = check_p2p(c, buf, count, dt, source, tag, true, &t);
    if (!rc && status) rc = check_buf(c->stream, status, 0, sizeof(mpixs_status), true);
    if (rc) return rc;
    if (c->sh->w->cfg.matching == 1) return MPIXS_ERR_COMM;   // sequence channels only
    World *w = c->sh->w;
    StreamObj *st = c->stream;
    if (hipStreamSynchronize(st->hs) != hipSuccess) return MPIXS_ERR_GPU;
    Channel *ch = get_channel(c, source, c->rank, tag, true);
    if (!ch) return MPIXS_ERR_NOMEM;
    const uint64_t k = ch->seq[1]++;
    Rec *rec;
    {
        std::lock_guard<std::mutex> g(ch->mu);
        rec = ch->at(k);
        rec->r.buf = buf;
        rec->r.count = count;
        rec->r.t = t;
        rec->r.bytes = int64_t(count) * t->L.size;
        rec->r.st = st;
        rec->r.rank = c->rank;
        rec->arrived.fetch_or(ARR_R, std::memory_order_release);
        host_notify(&rec->arrived);
    }
    rc = host_wait(w, &rec->arrived, [&] { return (rec->arrived.load(std::memory_order_acquire) & ARR_S) != 0; });
    if (rc) {
        rec_release(ch, rec);
        return rc;
    }
    Side S, R;
    {
        std::lock_guard<std::mutex> g(ch->mu);
        S = rec->s;
        R = rec->r;
    }
    const StatusVal sv = match_status(S, R, tag);
    rc = do_copy(w, st, S, R, sv, nullptr, 0, nullptr, 0, status, true);
    if (!rc && hipStreamSynchronize(st->hs) != hipSuccess) rc = MPIXS_ERR_GPU;
    rec->done_host.store(1, std::memory_order_release);
    host_notify(&rec->done_host);
    rec_release(ch, rec);
    return rc;
}

int mpixs_allreduce(const void *sendbuf, void *recvbuf, int count, mpixs_datatype dt, mpixs_op op,
                    mpixs_comm c) {
    int rc = check_allreduce(c, sendbuf, recvbuf, count, dt, op, true);
    if (rc) return rc;
    CommShared *sh = c->sh;
    World *w = sh->w;
    StreamObj *st = c->stream;
    if (hipStreamSynchronize(st->hs) != hipSuccess) return MPIXS_ERR_GPU;
    const uint64_t k = c->hcoll_seq++;
    const int n = sh->size;
    CollRec *rec;
    bool last;
    {
        std::lock_guard<std::mutex> g(sh->coll_mu);
        rec = coll_at(sh->hcolls, sh->hcoll_base, k, n);
        rec->in[c->rank] = sendbuf == MPIXS_IN_PLACE ? recvbuf : sendbuf;
        rec->out[c->rank] = recvbuf;
        if (rec->arrived == 0) {
            rec->count = count;
            rec->dtype = dt;
            rec->op = op;
        }
        last = ++rec->arrived == n;
    }
    if (last) {
        rc = do_reduce(w, st, rec, n, c->rank, nullptr, 0, nullptr, 0);
        if (!rc && hipStreamSynchronize(st->hs) != hipSuccess) rc = MPIXS_ERR_GPU;
        rec->done_host.store(1, std::memory_order_release);
        host_notify(&rec->done_host);
    } else {
        rc = host_wait(w, &rec->done_host, [&] { return rec->done_host.load(std::memory_order_acquire) != 0; });
    }
    if (rec->refs.fetch_sub(1) == 1) {
        std::lock_guard<std::mutex> g(sh->coll_mu);
        coll_collect(sh->hcolls, sh->hcoll_base);
    }
    return rc;
}

// ============================================================ diagnostics
int mpixs_world_get_stats(mpixs_world w, mpixs_stats *s) {
    if (!w || !s) return MPIXS_ERR_ARG;
    {
        std::lock_guard<std::mutex> g(w->prof_mu);
        std::vector<ProfPair> keep;
        for (auto &p : w->prof) {
            float ms = 0;
            hipError_t e = hipEventElapsedTime(&ms, p.e0, p.e1);
            if (e == hipErrorNotReady) {
                keep.push_back(p);
                continue;
            }
            if (e == hipSuccess) {
                if (p.kind == 0) {
                    w->timed_copy++;
                    w->copy_ms += ms;
                } else {
                    w->timed_reduce++;
                    w->reduce_ms += ms;
                }
            }
            (void)hipEventDestroy(p.e0);
            (void)hipEventDestroy(p.e1);
        }
        w->prof.swap(keep);
    }
    s->kernels_post = w->n_post.load();
    s->kernels_wait = w->n_wait.load();
    s->kernels_copy = w->n_copy.load();
    s->kernels_reduce = w->n_reduce.load();
    s->bytes_copied = w->bytes_copied.load();
    s->bytes_reduced = w->bytes_reduced.load();
    s->host_waits = w->host_waits.load();
    s->host_sleeps = w->host_sleeps.load();
    s->host_sleep_timeouts = w->host_sleep_timeouts.load();
    s->groups_planned = w->groups_planned.load();
    s->plan_ms = double(w->plan_ns.load()) * 1e-6;
    s->reductions_merged = w->reds_merged.load();
    s->channels_recycled = w->chans_recycled.load();
    s->eager_sends = w->n_eager.load();
    s->streams_recycled = w->streams_recycled.load();
    s->comm_lines_recycled = w->colls_recycled.load();
    s->timed_copy = w->timed_copy;
    s->copy_ms = w->copy_ms;
    s->timed_reduce = w->timed_reduce;
    s->reduce_ms = w->reduce_ms;
    return MPIXS_SUCCESS;
}

int mpixs_world_trace(mpixs_world w, mpixs_trace_event *events, int64_t max, int64_t *copied,
                      int64_t *total) {
    if (!w || !w->d_trace || !copied || !total || max < 0 || (max > 0 && !events))
        return MPIXS_ERR_ARG;
    *copied = 0;
    uint64_t head = 0;
    if (hipMemcpy(&head, w->d_trace_head, sizeof(head), hipMemcpyDeviceToHost) != hipSuccess)
        return MPIXS_ERR_GPU;
    *total = int64_t(head);
    // the last min(head, cap, max) events, oldest first
    const uint64_t kept = std::min<uint64_t>(head, w->trace_cap);
    const uint64_t n = std::min<uint64_t>(kept, uint64_t(max));
    if (n == 0) return MPIXS_SUCCESS;
    *copied = int64_t(n);
    std::vector<TraceEv> ring(static_cast<size_t>(w->trace_cap));
    if (hipMemcpy(ring.data(), w->d_trace, ring.size() * sizeof(TraceEv), hipMemcpyDeviceToHost) !=
        hipSuccess)
        return MPIXS_ERR_GPU;
    const double ns_per_tick = 1e6 / double(w->trace_rate_khz);
    for (uint64_t j = 0; j < n; ++j) {
        const TraceEv &e = ring[size_t((head - n + j) & (w->trace_cap - 1))];
        events[j].time_ns = uint64_t(double(e.ticks) * ns_per_tick);
        events[j].kind = e.kind;
        events[j].stream = e.stream;
        events[j].counter = e.counter;
        events[j].value = e.value;
    }
    return MPIXS_SUCCESS;
}

int mpixs_world_reset_stats(mpixs_world w) {
    if (!w) return MPIXS_ERR_ARG;
    mpixs_stats tmp;
    mpixs_world_get_stats(w, &tmp);
    w->n_post = 0;
    w->n_wait = 0;
    w->host_sleeps = 0;
    w->host_sleep_timeouts = 0;
    w->groups_planned = 0;
    w->plan_ns = 0;
    w->reds_merged = 0;
    w->chans_recycled = 0;
    w->n_eager = 0;
    w->streams_recycled = 0;
    w->colls_recycled = 0;
    w->n_copy = 0;
    w->n_reduce = 0;
    w->bytes_copied = 0;
    w->bytes_reduced = 0;
    w->host_waits = 0;
    std::lock_guard<std::mutex> g(w->prof_mu);
    w->timed_copy = w->timed_reduce = 0;
    w->copy_ms = w->reduce_ms = 0;
    return MPIXS_SUCCESS;
}

// Host-side introspection of the copy plan (no GPU work): the unit size
// and the source / destination address of every unit the copy kernel would
// move for a message of `nbytes` packed bytes.
int mpixs_debug_copy_plan(uint64_t sbuf, int scount, mpixs_datatype stype, uint64_t rbuf,
                          int rcount, mpixs_datatype rtype, int64_t nbytes, int64_t max_units,
                          uint64_t *src_addr, uint64_t *dst_addr, int *unit_bytes,
                          int64_t *nunits) {
    const TypeObj *ts = type_any(stype);
    const TypeObj *tr = type_any(rtype);
    if (!ts || !tr) return MPIXS_ERR_TYPE;
    if (!unit_bytes || !nunits) return MPIXS_ERR_ARG;
    // host copies of SEG tables, so uncommitted types can be planned too
    auto host_table = [](const TypeObj *t, std::vector<SegEnt> &tab) {
        int64_t pre = 0;
        for (auto &sg : t->L.segs) {
            tab.push_back(SegEnt{sg.first, pre});
            pre += sg.second;
        }
    };
    std::vector<SegEnt> tab_s, tab_r;
    host_table(ts, tab_s);
    host_table(tr, tab_r);
    // host copies of the granule tables too, so the plan takes the same
    // lookups as the kernels
    std::vector<uint32_t> lut_s, lut_r;
    TypeObj cs = *ts, cr = *tr;
    cs.table = tab_s.data();
    cs.nseg = int64_t(tab_s.size());
    cs.lut = (!cs.L.reg && seg_lut(cs.L, &lut_s, &cs.lut_shift)) ? lut_s.data() : nullptr;
    cr.table = tab_r.data();
    cr.nseg = int64_t(tab_r.size());
    cr.lut = (!cr.L.reg && seg_lut(cr.L, &lut_r, &cr.lut_shift)) ? lut_r.data() : nullptr;
    Side S, R;
    S.buf = reinterpret_cast<const void *>(sbuf);
    S.count = scount;
    S.t = &cs;
    S.bytes = int64_t(scount) * cs.L.size;
    R.buf = reinterpret_cast<const void *>(rbuf);
    R.count = rcount;
    R.t = &cr;
    R.bytes = int64_t(rcount) * cr.L.size;
    DMap ms, mr;
    int w = 16;
    uint64_t units = 0;
    plan_copy(S, R, nbytes, &ms, &mr, &w, &units);
    *unit_bytes = w;
    *nunits = int64_t(units);
    const uint64_t n = std::min<uint64_t>(units, uint64_t(std::max<int64_t>(max_units, 0)));
    auto addr = [&](const DMap &m, uint64_t u) -> uint64_t {
        switch (w * 4 + int(m.kind)) {
#define MPIXS_CASE(W)                                              \
    case W * 4 + MAP_CONTIG: return map_addr<MAP_CONTIG, W>(m, u); \
    case W * 4 + MAP_VEC: return map_addr<MAP_VEC, W>(m, u);       \
    case W * 4 + MAP_SEG: return map_addr<MAP_SEG, W>(m, u);
            MPIXS_CASE(1)
            MPIXS_CASE(2)
            MPIXS_CASE(4)
            MPIXS_CASE(8)
            MPIXS_CASE(16)
#undef MPIXS_CASE
        default: return ~uint64_t(0);
        }
    };
    for (uint64_t u = 0; u < n; ++u) {
        if (src_addr) src_addr[u] = addr(ms, u);
        if (dst_addr) dst_addr[u] = addr(mr, u);
    }
    return MPIXS_SUCCESS;
}

// Time the data kernel of one message: launch it `reps` times back to back
// on `hip_stream` between one pair of HIP events (no wait or signal kernels
// in between), synchronise, and return the average per launch.
int mpixs_debug_time_copy(void *hip_stream, const void *sbuf, int scount, mpixs_datatype stype,
                          void *rbuf, int rcount, mpixs_datatype rtype, int reps, double *avg_us,
                          int *unit_bytes) {
    const TypeObj *ts = type_lookup(stype);
    const TypeObj *tr = type_lookup(rtype);
    if (!ts || !tr) return MPIXS_ERR_TYPE;
    if (!avg_us || reps <= 0 || scount < 0 || rcount < 0) return MPIXS_ERR_ARG;
    Side S, R;
    S.buf = sbuf;
    S.count = scount;
    S.t = ts;
    S.bytes = int64_t(scount) * ts->L.size;
    R.buf = rbuf;
    R.count = rcount;
    R.t = tr;
    R.bytes = int64_t(rcount) * tr->L.size;
    const int64_t nbytes = std::min(S.bytes, R.bytes);
    DMap ms, mr;
    int wsz = 16;
    uint64_t units = 0;
    plan_copy(S, R, nbytes, &ms, &mr, &wsz, &units);
    if (unit_bytes) *unit_bytes = wsz;
    DevStream *scratch = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&scratch), sizeof(DevStream)) != hipSuccess)
        return MPIXS_ERR_NOMEM;
    hipStream_t hs = static_cast<hipStream_t>(hip_stream);
    int rc = MPIXS_SUCCESS;
    if (hipMemsetAsync(scratch, 0, sizeof(DevStream), hs) != hipSuccess) rc = MPIXS_ERR_GPU;
    CopyArgs a;
    std::memset(&a, 0, sizeof(a));
    a.src = ms;
    a.dst = mr;
    a.units = units;
    a.me = scratch;
    const uint64_t per_chunk = uint64_t(copy_block_units(false));
    const uint64_t nwg = std::max<uint64_t>(1, (units + per_chunk - 1) / per_chunk);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = MPIXS_ERR_GPU;
    if (!rc) rc = gpu_err(launch_copy(hs, a, wsz, int(nwg), false));   // warm
    if (!rc && hipEventRecord(e0, hs) != hipSuccess) rc = MPIXS_ERR_GPU;
    for (int i = 0; i < reps && !rc; ++i) rc = gpu_err(launch_copy(hs, a, wsz, int(nwg), false));
    if (!rc && hipEventRecord(e1, hs) != hipSuccess) rc = MPIXS_ERR_GPU;
    if (!rc && hipStreamSynchronize(hs) != hipSuccess) rc = MPIXS_ERR_GPU;
    float ms_total = 0;
    if (!rc && hipEventElapsedTime(&ms_total, e0, e1) != hipSuccess) rc = MPIXS_ERR_GPU;
    if (!rc) *avg_us = 1000.0 * double(ms_total) / reps;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(hs);
    (void)hipFree(scratch);
    return rc;
}

int mpixs_debug_time_batch(mpixs_batch b, void *hip_stream, int reps, double *avg_us,
                           int64_t *payload_bytes, int *workgroups) {
    if (!b || !b->p) return MPIXS_ERR_REQUEST;
    if (reps < 1 || !avg_us) return MPIXS_ERR_ARG;
    BatchPlan *P = b->p;
    if (payload_bytes) *payload_bytes = int64_t(P->bytes);
    if (workgroups) *workgroups = P->nwg;
    *avg_us = 0;
    const BatchArgs a = P->args;
    hipStream_t hs = static_cast<hipStream_t>(hip_stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = MPIXS_SUCCESS;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = MPIXS_ERR_GPU;
    if (!rc) rc = gpu_err(launch_batch(hs, a, P->nwg));   // warm
    if (!rc && hipEventRecord(e0, hs) != hipSuccess) rc = MPIXS_ERR_GPU;
    for (int i = 0; i < reps && !rc; ++i) rc = gpu_err(launch_batch(hs, a, P->nwg));
    if (!rc && hipEventRecord(e1, hs) != hipSuccess) rc = MPIXS_ERR_GPU;
    if (!rc && hipStreamSynchronize(hs) != hipSuccess) rc = MPIXS_ERR_GPU;
    float ms_total = 0;
    if (!rc && hipEventElapsedTime(&ms_total, e0, e1) != hipSuccess) rc = MPIXS_ERR_GPU;
    if (!rc) *avg_us = 1000.0 * double(ms_total) / reps;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(hs);
    return rc;
}

const char *mpixs_error_string(int err) {
    switch (err) {
    case MPIXS_SUCCESS: return "SUCCESS";
    case MPIXS_ERR_ARG: return "ERR_ARG";
    case MPIXS_ERR_COUNT: return "ERR_COUNT";
    case MPIXS_ERR_TYPE: return "ERR_TYPE";
    case MPIXS_ERR_RANK: return "ERR_RANK";
    case MPIXS_ERR_TAG: return "ERR_TAG";
    case MPIXS_ERR_COMM: return "ERR_COMM";
    case MPIXS_ERR_STREAM: return "ERR_STREAM";
    case MPIXS_ERR_REQUEST: return "ERR_REQUEST";
    case MPIXS_ERR_BUFFER: return "ERR_BUFFER";
    case MPIXS_ERR_NO_ENDPOINT: return "ERR_NO_ENDPOINT";
    case MPIXS_ERR_PENDING: return "ERR_PENDING";
    case MPIXS_ERR_NOMEM: return "ERR_NOMEM";
    case MPIXS_ERR_OP: return "ERR_OP";
    case MPIXS_ERR_TRUNCATE: return "ERR_TRUNCATE";
    case MPIXS_ERR_TIMEOUT: return "ERR_TIMEOUT";
    case MPIXS_ERR_ABORTED: return "ERR_ABORTED";
    case MPIXS_ERR_GPU: return "ERR_GPU";
    case MPIXS_ERR_INTERN: return "ERR_INTERN";
    default: return "ERR_UNKNOWN";
    }
}

}  // extern "C"
