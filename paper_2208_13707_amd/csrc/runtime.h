// Host-side objects of libmpixs.
#pragma once
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <cstdint>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/mpixs.h"
#include "mpixs_dev.h"

namespace mpixs {

// ------------------------------------------------------------- datatypes
// Layout of ONE element of a datatype as byte segments in packed order.
// REG: nblk segments of blen bytes, segment i at first + i * stride.
// SEG: an explicit list (adjacent segments merged).
struct Layout {
    int basic = 0;
    int esize = 0;
    int64_t size = 0;       // sum of entry sizes
    int64_t lb = 0, ub = 0, extent = 0;
    bool overlap = false;   // two entries share a byte
    bool reg = true;
    int64_t nblk = 0, blen = 0, stride = 0, first = 0;
    std::vector<std::pair<int64_t, int64_t>> segs;  // (offset, length)
    int64_t gcd = 0;        // gcd of every segment offset and length
    bool dense() const { return reg && nblk == 1; }
};

struct TypeObj {
    Layout L;
    bool predefined = false;
    bool committed = false;
    SegEnt *table = nullptr;   // SEG form: nseg entries in device memory
    int64_t nseg = 0;
    // SEG form: the segment holding each packed granule of 2^lut_shift bytes
    // of an element (device memory; nullptr for elements too large)
    uint32_t *lut = nullptr;
    uint32_t lut_shift = 0;
};

// Segment-lookup (granule) table of a SEG layout; false when too large.
bool seg_lut(const Layout &L, std::vector<uint32_t> *lut, uint32_t *shift);
// Returns nullptr unless `dt` names a committed datatype.
const TypeObj *type_lookup(mpixs_datatype dt);
// Any datatype, committed or not (nullptr if unknown).
const TypeObj *type_any(mpixs_datatype dt);
int basic_size(int basic);

// ----------------------------------------------------------------- world
struct World;
struct CommShared;

// Allocations a stream's enqueue calls have found accessible by the GPU
// (address ranges; host = pinned host memory, accepted for statuses only).
// Filled round-robin; used by the stream's one thread, so it needs no lock.
struct BufCache {
    static constexpr int N = 16;
    uintptr_t lo[N] = {}, hi[N] = {};
    bool host[N] = {};
    int next = 0;
};

struct StreamObj {
    World *w = nullptr;
    bool gpu = false;
    hipStream_t hs = nullptr;
    int endpoint = -1;
    DevStream *dev = nullptr;
    uint64_t tickets = 0;                 // tickets issued on dev->ticket
    std::atomic<int> comm_refs{0};
    BufCache bufs;
    uint64_t id = 0;                      // unique in the world (a freed stream's address may return)
};

struct Side {
    const void *buf = nullptr;
    int count = 0;
    const TypeObj *t = nullptr;
    int64_t bytes = 0;
    StreamObj *st = nullptr;
    int rank = -1;
    int idx = 0;                       // stream index (multiplex communicators)
};

enum : uint32_t { ARR_S = 1, ARR_R = 2 };

// Unit size and both address maps of a copy of `nbytes` packed bytes from
// S's typemap into R's.  seg_s / seg_r override the SEG tables (host-side
// planning of uncommitted types); nullptr uses the committed tables.
// tail != nullptr: a copy dense on both sides may leave its last nbytes mod W
// bytes to a byte tail (*tail), so that W follows the base addresses alone.
int plan_copy(const Side &S, const Side &R, int64_t nbytes, DMap *src, DMap *dst, int *wsz,
              uint64_t *units, uint32_t *tail = nullptr);

// Host record of message k of a channel: the first side to arrive stores
// its descriptor, the second side reads it and launches the copy.
struct Rec {
    std::atomic<uint32_t> arrived{0};
    std::atomic<int> copy_enq{0};      // second side launched the copy
    std::atomic<int> done_host{0};     // host-synchronised path: copy finished
    std::atomic<int> refs{2};
    Side s, r;
    StatusVal st{};
    // the message's device counters: block, and the value its ready / done
    // counters reach for this message (set with the record, under the
    // channel's lock)
    DevChan *d = nullptr;
    uint32_t didx = 0;
    uint64_t dv = 0;
    // eager send (complete on the sender's stream, the receiver's copy is
    // the message's last device use): the packed message in device staging
    // and the staging slot's host flag, set by that copy (none when empty)
    bool eager = false;
    uint8_t *stage = nullptr;
    int stage_flag = -1;
};

constexpr uint32_t kNoBlock = 0xffffffffu;

// A channel's device block is attached when a message needs it and may be
// handed back once the channel is quiescent (both sides have issued the same
// number of operations and the last of them has passed its wait on the
// device).  A block keeps its counter values across owners: an owner that
// attaches it at sequence number kbase with counters at most ebase uses the
// value ebase + (k - kbase) + 1 for its message k, above anything a former
// owner wrote, so the counters only ever grow.
struct Channel {
    DevChan *d = nullptr;
    uint32_t idx = kNoBlock;           // index of d in the world's pool
    uint64_t ebase = 0, kbase = 0;
    bool priv = false;                 // one message's channel (ordered-queue matching)
    uint64_t seq[2] = {0, 0};          // operations issued per side (under mu)
    std::mutex mu;
    std::deque<Rec *> recs;
    uint64_t base = 0;                 // sequence number of recs.front()
    // quiescent at drain_seq operations per side, once the device has
    // written drain_val to the block's release word (under the world's chan_mu)
    bool draining = false;
    uint64_t drain_seq = 0, drain_val = 0;
    CommShared *owner = nullptr;
    ~Channel();
    Rec *at(uint64_t k);               // caller holds mu
    void collect();                    // caller holds mu
    uint64_t dval(uint64_t k) const { return ebase + (k - kbase) + 1; }
};

struct CollRec {
    int arrived = 0;
    std::atomic<int> reduce_enq{0};
    std::atomic<int> posted{0};        // arrival kernels the non-reducing ranks have enqueued
    std::atomic<int> done_host{0};
    std::atomic<int> refs{0};
    const void *in[64] = {};
    void *out[64] = {};
    int count = 0, dtype = 0, op = 0;
};

// One operation recorded inside a group (see mpixs_group_start).
struct GOp {
    int kind = 0;                      // 0 send, 1 receive, 2 allreduce
    int peer = -1;
    int tag = 0;
    Side side;
    void *status = nullptr;            // receive status to write, or nullptr
    mpixs_request_s *req = nullptr;    // request to receive the status values
    // allreduce: input (the output for MPIXS_IN_PLACE), output, elements,
    // basic type and operation
    const void *red_in = nullptr;
    void *red_out = nullptr;
    int red_count = 0;
    int red_dtype = 0;
    int red_op = 0;
};

// One reduction of a group, planned for the launching rank's stream (the
// split reduce kernel: the group's wait and signal surround it).
struct RedPlan {
    ReduceArgs a{};
    int dtype = 0;
    int op = 0;
    int nwg = 0;
    bool vec = false;
    bool fixed = false;
    uint64_t bytes = 0;                // read + written, for the counters
};

// A group's allreduces merged into one reduce launch: all of one type and
// operator, each at most kMultiRedMaxBytes of input over all ranks, and no
// byte of any buffer shared by two of them (so their order cannot matter).
// Descriptors and the pointer table are copied next to the group's batch
// descriptors.
struct MultiRedPlan {
    bool on = false;
    bool nt = false;                   // nontemporal (large) launch
    int dtype = 0;
    int op = 0;
    int nwg = 0;
    uint32_t ninst = 0;
    uint64_t bytes = 0;                // read + written, for the counters
    std::vector<MultiRedDesc> desc;
    std::vector<const void *> ptrs;
};

struct BatchPlan;

struct GroupRec {
    int arrived = 0;
    int kind = 0;                       // 1: one-shot group_end, 2: persistent (group_end_init)
    bool mismatch = false;              // ranks ended the instance with different calls
    bool bad = false;                   // a persistent group left a request unwaited
    BatchPlan *batch = nullptr;         // group_end_init: the plan made by the last rank
    std::vector<std::vector<GOp>> ops;  // per rank
    std::vector<StreamObj *> streams;
    std::atomic<int> launched{0};
    std::atomic<int> posted{0};         // one-shot: arrival kernels the other ranks have enqueued
    int error = 0;
    std::atomic<int> refs{0};
    // Planning help: the planning rank may split the descriptor pass of a
    // large group into chunks; the other ranks, waiting for the launch,
    // take chunks until none is left (help_fn is set before help_on).
    std::function<void(size_t)> help_fn;
    size_t help_chunks = 0;
    std::atomic<int> help_on{0};
    std::atomic<size_t> help_next{0};
    std::atomic<size_t> help_done{0};
};

// A persistent batch: a group planned once, run by every start.  Device
// memory holds the counters (arrive[q] at word 16q, done at word 16n, all
// counting runs), the descriptors and the workgroup starts.
struct BatchPlan {
    World *w = nullptr;
    int n = 0;
    int leader = -1;                    // the rank whose stream launches the batch kernel
    uint8_t *d_mem = nullptr;
    bool static_mem = false;            // d_mem is the device's static region (not freed)
    int device = 0;
    uint64_t static_gen = 0;            // the region's contents this plan wrote
    uint64_t *d_ctr = nullptr;
    BatchArgs args{};
    RelWaitArgs lwait{};                // leader: every other rank arrived for this run
    SignalArgs sig{};                   // leader, after the batch kernel: done + 1
    int nwg = 0;
    uint64_t nmsg = 0, bytes = 0;
    std::vector<RedPlan> reds;          // allreduces of the group, after the batch kernel
    MultiRedPlan mred;                  // or all of them in one launch
    MultiRedArgs margs{};               // its descriptors in d_mem
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> post_ev;    // batch_sync = 1: per rank, recorded at its arrival
    hipEvent_t done_ev = nullptr;       // batch_sync = 1: recorded after the batch kernel
    std::unique_ptr<std::atomic<uint64_t>[]> posted;   // runs whose arrival rank q has enqueued
    std::atomic<uint64_t> launched{0};                  // runs the leader has enqueued
    std::atomic<int> launch_err{0};
    std::atomic<int> refs{0};
    ~BatchPlan();
};

// The static region for persistent batches planned without allocating
// (mpixs_group_end_init_static), one per GPU.  static_batch_setup finds this
// device's copy (called once per device, with it current, when a world is
// created there); static_batch_region hands it to a new plan (ERR_NOMEM when
// the plan needs more, ERR_GPU without a region) and counts its owners;
// static_batch_current tells whether a plan still owns it.
constexpr size_t kStaticBatchBytes = size_t(4) << 20;
void static_batch_setup(int device);
int static_batch_region(int device, size_t bytes, uint8_t **ptr, uint64_t *gen);
bool static_batch_current(int device, uint64_t gen);

struct CreateRec {
    int arrived = 0;
    int left = 0;
    CommShared *sh = nullptr;
};

// Collective lines of a freed communicator: reusable once every stream its
// ranks used is idle or freed (a stream is freed only when idle), so no
// kernel of the old communicator can still write them; a new owner
// continues the instance numbers from the floors, so its counter targets
// stay above the values already there.
struct CollLines {
    size_t off = 0, words = 0;
    uint64_t floor_coll = 0, floor_group = 0;
    std::vector<std::pair<StreamObj *, uint64_t>> users;   // stream and its id
};

// Ordered-queue matching (mpixs_config.matching = 1): per destination rank,
// the receives posted and the sends enqueued that have not met a partner
// yet, each with its own one-message channel.
struct QOp {
    Channel *ch = nullptr;
    Rec *rec = nullptr;
    int src = 0;                       // a send's source; a receive's source or ANY_SOURCE
    int src_idx = 0;                   // a send's stream index; a receive's or ANY_INDEX
    int tag = 0;                       // a send's tag; a receive's tag or ANY_TAG
};

struct MatchQueue {
    std::mutex mu;
    std::deque<QOp> unexpected;        // sends, in enqueue order
    std::deque<QOp> posted;            // receives, in post order
};

// Working arrays of group planning, kept by a communicator so that their
// memory is reused from one group instance to the next.
struct PlanScratch {
    struct Slot {
        uint64_t key;
        uint32_t chan;
    };
    std::vector<Slot> table;            // open addressing: channel key -> channel
    std::vector<uint32_t> chan_of;      // channel of every grouped operation
    std::vector<uint32_t> nsend, nrecv, first, fill_s, fill_r;
    std::vector<GOp *> s_of, r_of;      // pair i: its send and its receive
    std::vector<BatchDesc> descs;
    std::vector<BatchStart> starts;
    std::vector<uint64_t> part;         // per descriptor chunk: tiles, bytes
    size_t nstarts = 0;                 // workgroup starts of the last plan
    std::vector<RedPlan> reds;         // the group's allreduces, in order
    MultiRedPlan mred;                 // the same, merged when allowed
};

struct CommShared {
    World *w = nullptr;
    int size = 0;
    uint32_t id = 0;
    std::vector<StreamObj *> streams;
    std::mutex dir_mu;
    std::unordered_map<uint64_t, Channel *> dir;
    std::mutex coll_mu;
    std::deque<CollRec *> colls;
    uint64_t coll_base = 0;
    std::deque<CollRec *> hcolls;      // host-synchronised allreduce instances
    uint64_t hcoll_base = 0;
    uint64_t *d_coll = nullptr;        // arrive[q] at 16*q, done at 16*size
    uint64_t *d_grp = nullptr;         // groups: arrive[q] at 16*q, done at 16*size
    std::mutex grp_mu;
    std::deque<GroupRec *> groups;
    std::mutex plan_mu;                // one group plan at a time uses `plan`
    PlanScratch plan;
    uint64_t group_base = 0;
    std::mutex create_mu;
    std::map<uint64_t, CreateRec> creates;
    std::atomic<int> handles{0};
    std::unique_ptr<MatchQueue[]> mq;  // ordered-queue matching, one per endpoint
    // multiplex communicators (§3.5): every rank attaches several streams;
    // endpoint (rank, index) has queue ep_base[rank] + index
    bool multiplex = false;
    std::vector<std::vector<StreamObj *>> mst;
    std::vector<int> ep_base;
    bool ep_ready = false;             // under create_mu of the parent
    // device collective lines (d_coll, d_grp): offset and words in the
    // world's collective pool, the instance numbers they start from, and
    // what the freeing ranks leave for their reuse (under free_mu)
    size_t coll_off = 0, coll_words = 0;
    uint64_t floor_coll = 0, floor_group = 0;
    std::mutex free_mu;
    std::vector<std::pair<StreamObj *, uint64_t>> users;
    uint64_t max_coll = 0, max_group = 0;
    ~CommShared();
};

}  // namespace mpixs

struct mpixs_info_s {
    std::map<std::string, std::string> kv;
};

struct mpixs_stream_s : mpixs::StreamObj {};

struct mpixs_comm_s {
    mpixs::CommShared *sh = nullptr;
    int rank = -1;
    mpixs::StreamObj *stream = nullptr;
    std::unordered_map<uint64_t, mpixs::Channel *> cache;
    uint64_t coll_seq = 0, hcoll_seq = 0, create_seq = 0, group_seq = 0;
    std::atomic<int> pending{0};
    bool world_handle = false;
    bool in_group = false;
    std::vector<mpixs::GOp> gops;
    std::vector<mpixs::StreamObj *> mstreams;   // multiplex: local streams by index
};

struct mpixs_request_s {
    mpixs_comm_s *comm = nullptr;
    mpixs::Channel *ch = nullptr;
    mpixs::Rec *rec = nullptr;
    uint64_t k = 0;
    int side = 0;                      // 0 send, 1 receive
    bool second = false;               // this side launched the copy itself
    bool grouped = false;              // recorded in a group: complete at group_end
    size_t gop = 0;                    // index in the comm's recorded operations
    mpixs::StatusVal st{};
    mpixs::StreamObj *stream = nullptr; // the stream the request was enqueued on
};

struct mpixs_batch_s {
    mpixs::BatchPlan *p = nullptr;
    mpixs_comm_s *comm = nullptr;
    int rank = -1;
    uint64_t runs = 0;                 // runs this rank has enqueued
};

namespace mpixs {

struct ProfPair {
    hipEvent_t e0, e1;
    int kind;                           // 0 copy, 1 reduce
};

struct World {
    int nranks = 0;
    int device = 0;
    mpixs_config cfg{};
    char *d_pool = nullptr;
    DevStream *d_streams = nullptr;
    int stream_cap = 0;
    std::atomic<int> stream_next{0};
    DevChan *d_chans = nullptr;
    uint32_t chan_cap = 0;
    std::atomic<uint32_t> chan_next{0};
    uint64_t *d_coll = nullptr;
    size_t coll_words = 0;
    std::atomic<size_t> coll_next{0};
    // block recycling: channel blocks (index, counter floor) ready for a new
    // owner; channels whose block may be handed back once the device has
    // written the release word; blocks of dead one-message channels waiting
    // for their release word; stream blocks returned by mpixs_stream_free
    // (block index, ticket count); collective lines of freed communicators
    std::mutex chan_mu;
    std::vector<std::pair<uint32_t, uint64_t>> chan_free;
    std::vector<Channel *> chan_drain;
    std::vector<std::pair<uint32_t, uint64_t>> chan_limbo;
    uint64_t *h_rel = nullptr;         // host-pinned release word per channel block
    std::vector<std::pair<int, uint64_t>> stream_free;   // under ep_mu
    std::mutex coll_mu;
    std::vector<CollLines> coll_free;
    std::atomic<uint64_t> next_stream_id{1};
    std::atomic<uint64_t> chans_recycled{0}, streams_recycled{0}, colls_recycled{0};
    uint32_t *h_abort = nullptr;       // host-pinned, read by device waits
    std::atomic<int> aborted{0};
    uint64_t timeout_ticks = 0;
    // endpoints: finite, shared round-robin under policy 1
    std::mutex ep_mu;
    std::vector<int> ep_users;
    int ep_rr = 0;
    std::atomic<uint32_t> next_comm_id{1};
    CommShared *world_sh = nullptr;
    std::vector<mpixs_comm_s *> world_handles;
    std::mutex reg_mu;
    std::set<StreamObj *> streams;
    std::atomic<int> live_comms{0};
    // statistics
    std::atomic<uint64_t> n_post{0}, n_wait{0}, n_copy{0}, n_reduce{0};
    std::atomic<uint64_t> bytes_copied{0}, bytes_reduced{0}, host_waits{0};
    std::atomic<uint64_t> host_sleeps{0}, host_sleep_timeouts{0};
    std::atomic<uint64_t> groups_planned{0}, plan_ns{0};
    std::atomic<uint64_t> reds_merged{0};   // allreduces run inside a merged reduce launch
    // host-pinned (coherent) ring of batch descriptor tables; an entry is
    // recycled once the batch's signal kernel has set its flag
    struct ArenaUse {
        size_t off, bytes;
        int flag;
    };
    std::mutex arena_mu;
    char *h_arena = nullptr;
    size_t arena_bytes = 0;
    size_t arena_head = 0;
    std::deque<ArenaUse> arena_live;
    uint32_t *h_flags = nullptr;
    int nflags = 0;
    std::vector<int> free_flags;
    // device staging ring of eager sends, recycled in order like the batch
    // arena: a slot is free again once the receiver's copy has set its flag
    struct StageRing {
        std::mutex mu;
        uint8_t *base = nullptr;   // device memory
        size_t bytes = 0, head = 0;
        std::deque<ArenaUse> live;
        uint32_t *flags = nullptr;   // host-pinned, coherent
        int nflags = 0;
        std::vector<int> free_flags;
    } stage;
    std::atomic<uint64_t> n_eager{0};
    // device trace ring (trace_events > 0): events and the slot counter
    TraceEv *d_trace = nullptr;
    uint64_t *d_trace_head = nullptr;
    uint64_t trace_cap = 0;
    int trace_rate_khz = 0;
    // eager messages whose receive is not enqueued yet: each holds its
    // channel's block until then, so they may take at most half the pool
    // (the rest serves rendezvous, whose waits bound what is in flight)
    std::atomic<int64_t> eager_held{0};
    std::mutex prof_mu;
    std::vector<ProfPair> prof;
    uint64_t timed_copy = 0, timed_reduce = 0;
    double copy_ms = 0, reduce_ms = 0;
};

}  // namespace mpixs

struct mpixs_world_s : mpixs::World {};
