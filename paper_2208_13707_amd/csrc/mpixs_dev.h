// Device-side data layout and kernel argument blocks of libmpixs.
//
// Everything the kernels read arrives either in the kernel argument block
// (maps, pointers, counts: the host knows both sides of a matched message
// when it launches the copy) or in the world's device pool, which holds
//   - one 64-byte "channel" block per (communicator, source, destination,
//     tag): two ready counters (one per side) and a done counter.  These
//     monotone counters are the device matching table: the k-th operation
//     of a side on a channel posts ready = k+1 when its stream reaches it,
//     and the copy of message k publishes done = k+1 (§2.1: matching order
//     is per channel, in issue order);
//   - one 128-byte block per stream (first asynchronous error, fatal flag,
//     completion ticket counter);
//   - per communicator, one arrive counter per rank and a done counter for
//     collectives.
#pragma once
#include <stdint.h>

#ifndef MPIXS_HD
#if defined(__HIPCC__)
#define MPIXS_HD __host__ __device__
#else
#define MPIXS_HD
#endif
#endif

namespace mpixs {

// ------------------------------------------------------------ fast division
// Division of a 32-bit n by an invariant d >= 1 with one multiply-high
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, §4): with l = ceil(log2 d) and
// m = floor(2^32 * (2^l - d) / d) + 1, n / d = (mulhi(n, m) + n) >> l,
// the sum taken in 64 bits.
struct FastDiv {
    uint32_t d;
    uint32_t m;
    uint32_t l;
    uint32_t pad;
};

static inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    f.l = l;
    f.m = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
    f.pad = 0;
    return f;
}

MPIXS_HD static inline uint32_t fd_div(uint32_t n, const FastDiv &f) {
    uint32_t t = uint32_t((uint64_t(n) * f.m) >> 32);
    return uint32_t((uint64_t(t) + n) >> f.l);
}

// ---------------------------------------------------------------- typemaps
enum MapKind : uint32_t { MAP_CONTIG = 0, MAP_VEC = 1, MAP_SEG = 2 };

// One segment of a flattened typemap: byte offset from the start of a copy
// (the buffer address plus copy * extent) and the packed bytes before it.
struct SegEnt {
    int64_t off;
    int64_t pre;
};

// Map from packed unit u (units of W bytes) of one side of a message to the
// byte address holding it.
//   CONTIG: base + u * W
//   VEC:    c = u / upc, r = u % upc, b = r / bu, o = r % bu
//           base + c * s_copy + b * s_blk + o * W
//   SEG:    c = u / upc, rb = (u % upc) * W, i = last segment with pre <= rb
//           (lut[rb >> shift] when the type has a granule table, else a
//           binary search of the prefixes)
//           base + c * s_copy + seg[i].off + (rb - seg[i].pre)
struct DMap {
    uint64_t base;
    uint32_t kind;
    uint32_t upc;     // units per copy (VEC, SEG)
    uint32_t bu;      // VEC: units per block; SEG: log2 of the granule of lut
    uint32_t nseg;    // segments per copy (SEG)
    int64_t s_copy;   // bytes between copies
    union {
        int64_t s_blk;          // VEC: bytes between blocks
        const uint32_t *lut;    // SEG: segment of each packed granule, or nullptr
    };
    FastDiv d_upc;
    FastDiv d_bu;
    const SegEnt *seg;  // SEG table (nseg entries), in device memory
};

template <int K, int W>
MPIXS_HD inline uint64_t map_addr(const DMap &m, uint64_t u) {
    if constexpr (K == MAP_CONTIG) {
        return m.base + u * W;
    } else if constexpr (K == MAP_VEC) {
        const uint32_t u32 = uint32_t(u);
        const uint32_t c = fd_div(u32, m.d_upc);
        const uint32_t r = u32 - c * m.upc;
        const uint32_t b = fd_div(r, m.d_bu);
        const uint32_t o = r - b * m.bu;
        return m.base + uint64_t(int64_t(c) * m.s_copy + int64_t(b) * m.s_blk) + uint64_t(o) * W;
    } else {
        const uint32_t u32 = uint32_t(u);
        const uint32_t c = fd_div(u32, m.d_upc);
        const int64_t rb = int64_t(u32 - c * m.upc) * W;
        // last segment whose packed prefix is <= rb: one load of the granule
        // table (units never straddle a granule), else a binary search
        uint32_t lo = 0;
        if (m.lut) {
            lo = m.lut[uint64_t(rb) >> m.bu];
        } else {
            uint32_t hi = m.nseg;
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (m.seg[mid].pre <= rb) lo = mid; else hi = mid;
            }
        }
        const SegEnt e = m.seg[lo];
        return m.base + uint64_t(int64_t(c) * m.s_copy + e.off + (rb - e.pre));
    }
}

// ------------------------------------------------------------ device state
struct alignas(64) DevChan {
    uint64_t ready[2];    // [0]: sender side, [1]: receiver side
    uint64_t done;
    uint64_t pad[5];
};

// One event of the device trace (the public record, with ticks in place of
// nanoseconds).
struct TraceEv {
    uint64_t ticks;
    uint32_t kind;
    uint32_t stream;
    uint64_t counter;
    uint64_t value;
};

struct alignas(128) DevStream {
    uint32_t first_error;  // first asynchronous error of this stream (0: none)
    uint32_t fatal;        // non-zero: a wait gave up; later data movement is skipped
    uint64_t ticket;       // completion tickets of multi-workgroup kernels
    // the world's trace ring (written once at world creation); kernels read
    // it only when their arguments ask for an event
    TraceEv *trace;
    uint64_t *trace_head;
    uint32_t trace_mask;
    uint32_t slot;         // this block's index
    uint64_t pad[11];
};

// -------------------------------------------------------------- arguments
struct StatusVal {
    int32_t source;
    int32_t tag;
    int32_t error;
    int32_t source_index;   // sender's stream index (multiplex communicators), else 0
    int64_t count_bytes;
};

struct WaitCtl {
    const uint32_t *abort;           // host-pinned abort word of the world
    uint64_t timeout_ticks;          // wall-clock ticks before a wait gives up
};

// Up to 64 (pointer, target) pairs: wait until *ptr >= target for each.
// A lane whose rel_idx is nonzero is the last device user of channel block
// rel_idx - 1: once its wait has passed it writes its target to that
// block's host-pinned release word, which lets the host hand the block on.
struct WaitArgs {
    const uint64_t *ptr[64];
    uint64_t target[64];
    int32_t n;
    uint32_t trace;         // trace kind each passing lane records (0: none)
    WaitCtl ctl;
    DevStream *me;          // stream the kernel runs on
    void *status;           // optional receive status to write after the wait
    StatusVal st;
    uint64_t *rel_base;     // host-pinned release words, one per channel block
    uint32_t rel_idx[64];
};

struct CopyArgs {
    DMap src;
    DMap dst;
    uint64_t units;               // W-byte units to copy
    // fused wait (nullptr: the stream already waited)
    const uint64_t *wait_ptr;
    uint64_t wait_target;
    WaitCtl ctl;
    // completion
    uint64_t *done_ptr;           // nullptr: no channel to signal
    uint64_t done_val;
    DevStream *me;
    uint64_t ticket_last;         // ticket value that the last workgroup draws
    void *status;                 // optional receive status
    StatusVal st;
    int32_t set_error;            // copy st.error into me->first_error
    uint32_t trace;               // fused: record MATCH after the wait, DONE at publish
    // fused only, after done: a host-pinned word set to 1 (the host may
    // recycle what the kernel read), and a host-pinned release word set to
    // rel_val (the kernel was the last device use of a channel block)
    uint32_t *host_flag;
    uint64_t *rel_word;
    uint64_t rel_val;
};

// Completion of a message or collective after the stream's data kernel:
// optional status and sticky error, then done = val, then (optional) a
// host-pinned word set to 1 so the host may recycle what the kernel read,
// and (optional) a channel block's host-pinned release word set to rel_val.
struct SignalArgs {
    uint64_t *done_ptr;
    uint64_t done_val;
    DevStream *me;
    void *status;
    StatusVal st;
    int32_t set_error;
    int32_t inc;            // nonzero: done = done + 1 (single writer), done_val unused
    uint32_t *host_flag;
    uint64_t *rel_word;
    uint64_t rel_val;
    uint32_t trace;         // record DONE
    uint32_t pad;
};

// Relative wait of a persistent batch: lane q < n (bit q of skip clear)
// waits until ptr0[q * stride] >= *base + delta.  Targets are read on the
// device, so the same arguments serve every run of the batch.
struct RelWaitArgs {
    const uint64_t *ptr0;
    const uint64_t *base;
    uint64_t delta;
    uint64_t skip;
    uint32_t n;
    uint32_t stride;        // in uint64_t words
    WaitCtl ctl;
    DevStream *me;
    uint32_t trace;         // record MATCH per passing lane
    uint32_t pad;
};

// ----------------------------------------------------------------- batches
// One message of a batch (in host-pinned memory for a one-shot group, in
// device memory for a persistent batch).  It is cut into tiles of
// tile * 16 bytes (tile = 256 .. 4096, the same for the whole batch), that
// is tile * 16 / w units of w bytes, so tiles are balanced by bytes; a
// message dense on both sides may end in a byte tail of fewer than w bytes,
// copied with its last tile.  The workgroup that runs a message's tile 0
// also writes the message's receive status.
constexpr uint32_t BATCH_TILE_DEFAULT = 256;
constexpr uint32_t BATCH_TILE_MIN = 256;
constexpr uint32_t BATCH_TILE_MAX = 4096;

struct alignas(16) BatchDesc {
    DMap src;
    DMap dst;
    uint64_t units;
    uint32_t w;             // unit bytes: 1, 2, 4, 8 or 16
    uint32_t ntiles;        // max(1, ceil(units / (tile * 16 / w)))
    void *status;           // receive status or nullptr
    DevStream *rstream;     // receiver's stream block (sticky error)
    StatusVal st;
    uint32_t tail;          // bytes after the units (both maps dense), < w
    uint32_t pad;
};

// First tile of a workgroup: message index and tile within that message.
struct BatchStart {
    uint32_t msg;
    uint32_t tile;
};

static_assert(sizeof(BatchDesc) % 16 == 0, "descriptors are fetched in 16-byte words");
static_assert(sizeof(DevStream) == 128, "one stream block per 128 bytes");

struct BatchArgs {
    const BatchDesc *desc;
    const BatchStart *start;
    uint32_t nmsg;
    uint32_t extra;         // workgroups b < extra run base + 1 tiles
    uint64_t base;          // tiles per workgroup
    DevStream *me;
    uint32_t tile;          // units per tile
    uint32_t nt;            // nonzero: nontemporal loads and stores
};

enum RedOp : int32_t { OP_SUM = 1, OP_PROD = 2, OP_MIN = 3, OP_MAX = 4 };

struct ReduceArgs {
    const void *in[64];
    void *out[64];
    int32_t n;
    int32_t me_rank;
    uint64_t count;               // elements
    // fused wait on the other ranks' arrive counters (nullptr: waited already)
    const uint64_t *arrive;
    uint64_t arrive_target;
    WaitCtl ctl;
    uint64_t *done_ptr;
    uint64_t done_val;
    DevStream *me;
    uint64_t ticket_last;
    uint32_t trace;               // fused: record MATCH after the arrivals, DONE at publish
    uint32_t pad;
};

// Several small reductions of one element type and operator in one launch
// (a group's allreduces).  Instance i owns workgroups [first_wg, next
// instance's first_wg); its rank buffers are ptrs[ptr .. ptr+n) (inputs) and
// ptrs[ptr+n .. ptr+2n) (outputs).  No instance's buffers overlap another's.
struct MultiRedDesc {
    uint64_t count;         // elements
    uint32_t first_wg;
    uint32_t ptr;
    uint32_t n;
    uint32_t vec;           // nonzero: every buffer 16-byte aligned
};

struct MultiRedArgs {
    const MultiRedDesc *desc;
    const void *const *ptrs;
    uint32_t ninst;
    DevStream *me;
};

}  // namespace mpixs
