/*
 * mpixs.h -- stream-ordered point-to-point and allreduce traffic enqueued on
 * HIP streams of one MI355X (gfx950).
 *
 * This is the C ABI of libmpixs.so.  It implements the "MPIX stream" idea of
 * Zhou, Raffenetti, Guo and Thakur, "MPIX Stream: An Explicit Solution to
 * Hybrid MPI+X Programming" (EuroMPI/USA'22): a stream object names a serial
 * execution context (here: a HIP stream), a stream communicator attaches one
 * such context per rank, and enqueue calls put point-to-point and collective
 * operations on that context, to run there in order, with no host
 * synchronisation.
 *
 * Ranks are host threads of one process sharing one GPU: a "world" of N
 * ranks stands in for MPI_COMM_WORLD, and every rank thread calls the
 * functions below with its own communicator handle.  Payload work (datatype
 * gather/scatter, the copy into the matched receive buffer, the reduction)
 * runs in the library's HIP kernels on the streams.
 *
 * General rules
 *  - Every function returns MPIXS_SUCCESS (0) or an error class below.  An
 *    error returned by an enqueue call is synchronous and has no side
 *    effect: nothing was enqueued and no matching sequence advanced.
 *  - Errors found while an operation runs on the GPU (truncation, datatype
 *    signature mismatch, a device wait that timed out or was aborted) are
 *    written to the receive status (if one was given) and to the stream's
 *    sticky error word, read with mpixs_stream_get_error().
 *  - Objects (world, info, stream, comm, request, derived datatypes) are
 *    owned by the library; *_free calls set the caller's handle to NULL/0.
 *  - Buffers and statuses are owned by the caller and must be device
 *    memory of the world's GPU (hipMalloc, torch tensors) or, for statuses
 *    only, host memory allocated with hipHostMalloc.  They must stay valid
 *    and untouched until the stream has passed the operation, as with any
 *    enqueued GPU work.
 *  - The hipStream_t given to mpixs_stream_create() stays owned by the
 *    caller and must outlive the mpixs_stream.
 *  - Threading: a stream, and every communicator built on it, is used by one
 *    host thread at a time (the serial-context contract, §3.1).  World,
 *    info and datatype calls are thread-safe.
 */
#ifndef MPIXS_H
#define MPIXS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ errors */
enum {
    MPIXS_SUCCESS = 0,
    MPIXS_ERR_ARG = 1,          /* invalid argument (NULL handle, size out of range) */
    MPIXS_ERR_COUNT = 2,        /* negative count; a message of 2^32 bytes or more whose
                                   datatype is not dense (its device unit index is 32-bit) */
    MPIXS_ERR_TYPE = 3,         /* bad or uncommitted datatype; overlapping receive type;
                                   signature mismatch (asynchronous) */
    MPIXS_ERR_RANK = 4,         /* peer rank out of range, or a wildcard where none is allowed */
    MPIXS_ERR_TAG = 5,          /* negative tag, or a wildcard where none is allowed */
    MPIXS_ERR_COMM = 6,         /* communicator has no local GPU stream (§3.4) */
    MPIXS_ERR_STREAM = 7,       /* waitall over requests of different streams (§3.4) */
    MPIXS_ERR_REQUEST = 8,      /* NULL or foreign request */
    MPIXS_ERR_BUFFER = 9,       /* buffer or status not accessible by the GPU */
    MPIXS_ERR_NO_ENDPOINT = 10, /* stream pool exhausted (§3.1) */
    MPIXS_ERR_PENDING = 11,     /* free of an object with operations in flight (§3.1) */
    MPIXS_ERR_NOMEM = 12,       /* device tables or host memory exhausted */
    MPIXS_ERR_OP = 13,          /* unknown reduction operation */
    MPIXS_ERR_TRUNCATE = 14,    /* message longer than the receive buffer (asynchronous) */
    MPIXS_ERR_TIMEOUT = 15,     /* a host or device wait gave up */
    MPIXS_ERR_ABORTED = 16,     /* mpixs_world_abort() was called */
    MPIXS_ERR_GPU = 17,         /* a HIP runtime call failed */
    MPIXS_ERR_INTERN = 18
};

/* ----------------------------------------------------------------- handles */
typedef struct mpixs_world_s *mpixs_world;
typedef struct mpixs_info_s *mpixs_info;
typedef struct mpixs_stream_s *mpixs_stream;
typedef struct mpixs_comm_s *mpixs_comm;
typedef struct mpixs_request_s *mpixs_request;
typedef struct mpixs_batch_s *mpixs_batch;     /* a persistent group (one handle per rank) */
typedef int32_t mpixs_datatype;
typedef int32_t mpixs_op;

#define MPIXS_INFO_NULL ((mpixs_info)0)
#define MPIXS_STREAM_NULL ((mpixs_stream)0)
#define MPIXS_REQUEST_NULL ((mpixs_request)0)
#define MPIXS_DATATYPE_NULL ((mpixs_datatype)0)
#define MPIXS_ANY_SOURCE (-2)
#define MPIXS_ANY_TAG (-1)
#define MPIXS_ANY_INDEX (-3)    /* any stream index (multiplex communicators, §3.5) */
#define MPIXS_IN_PLACE ((const void *)1)

/* basic datatypes (homogeneous; derived types are built from one of them) */
#define MPIXS_UINT8 ((mpixs_datatype)1)
#define MPIXS_INT8 ((mpixs_datatype)2)
#define MPIXS_INT32 ((mpixs_datatype)3)
#define MPIXS_FLOAT32 ((mpixs_datatype)4)
#define MPIXS_INT64 ((mpixs_datatype)5)
#define MPIXS_FLOAT64 ((mpixs_datatype)6)

/* reduction operations */
#define MPIXS_SUM ((mpixs_op)1)
#define MPIXS_PROD ((mpixs_op)2)
#define MPIXS_MIN ((mpixs_op)3)
#define MPIXS_MAX ((mpixs_op)4)

/* Receive status (the MPI_Status of §3.4's receive calls).  count_bytes is
 * the number of bytes written into the receive buffer.  Pass NULL to ignore. */
typedef struct {
    int32_t source;
    int32_t tag;
    int32_t error;
    int32_t source_index;       /* sender's stream index on a multiplex communicator, else 0 */
    int64_t count_bytes;
} mpixs_status;

/* World configuration.  Zero fields take the default in brackets. */
typedef struct {
    int32_t max_streams;      /* stream (endpoint) pool size [256]; the pool is finite
                                 as network endpoints are (§2.2, §3.1) */
    int32_t endpoint_policy;  /* 0: stream_create fails when the pool is empty;
                                 1: share endpoints round-robin (§3.1) [0] */
    int32_t fuse_max_bytes;   /* messages (and allreduces, counting all ranks' inputs) up
                                 to this size wait and copy in one kernel of at most 32
                                 workgroups; larger ones use a one-wave wait kernel, a
                                 full-grid data kernel and a signal kernel [65536];
                                 -1: never fuse */
    int32_t timeout_ms;       /* host waits for a peer's enqueue, and device waits for a
                                 peer's stream, give up after this [30000] */
    int32_t max_channels;     /* device matching-table capacity in channels [1<<20] */
    int32_t profile;          /* 1: time copy and reduce kernels with HIP events */
    int32_t max_collectives;  /* device collective-slot capacity [4096] */
    int32_t batch_arena_mib;  /* host-pinned memory for batch descriptors, MiB [64]; a
                                 one-shot group in flight holds 224 bytes per message
                                 and 8 per batch_max_wg workgroup (a larger group
                                 fails with MPIXS_ERR_NOMEM) */
    int32_t batch_tile;       /* tile of the batch kernel in 16-byte units: 256, 512, 1024,
                                 2048 or 4096 [256]; other values: MPIXS_ERR_ARG */
    int32_t batch_max_wg;     /* workgroups of one batch kernel, at most [32768] */
    int32_t batch_graph;      /* persistent batches: 1 replays the launching rank's part
                                 of a run (wait, batch kernel, signal) as one HIP graph,
                                 0 launches the three kernels one by one [0] */
    int32_t batch_nontemporal; /* batch kernel loads and stores: 0 nontemporal for groups
                                 of at least 64 MiB of payload, 1 always, 2 never [0] */
    int32_t matching;         /* point-to-point matching (§2.1): 0 sequence pairing per
                                 (comm, source, destination, tag) channel, wildcards
                                 rejected; 1 ordered queues per destination, receives may
                                 use MPIXS_ANY_SOURCE / MPIXS_ANY_TAG [0] */
    int32_t batch_sync;       /* persistent batches: how a run's arrivals and completion
                                 are ordered across the ranks' streams: 0 device counters
                                 (an arrival kernel on every rank, a wait kernel and a
                                 signal kernel around the batch kernel), 1 HIP events
                                 (hipEventRecord / hipStreamWaitEvent, no extra kernels;
                                 not with batch_graph = 1) [0] */
    int32_t eager_max_bytes;  /* a blocking send whose receive is not yet enqueued, of
                                 at most eager_max_bytes, is packed into device staging
                                 on the sender's stream and completes there (eager; an
                                 empty one only posts), so the call returns at once;
                                 larger ones, or all when staging or half the matching
                                 table is held by eager messages, wait for their receive
                                 to be enqueued (rendezvous) [65536]; -1: never eager */
    int32_t eager_arena_mib;  /* device staging of eager sends, MiB [64] */
    int32_t trace_events;     /* capacity of the device event trace (rounded up to a power
                                 of two, at most 2^24; the newest events overwrite the
                                 oldest), read by mpixs_world_trace; 0: no tracing [0] */
    int32_t reserved[3];
} mpixs_config;

/* ------------------------------------------------------------------ tracing
 * With mpixs_config.trace_events > 0 the kernels record, in a device ring,
 * when each step of an operation happens on the GPU (§3.4: the operations
 * run on the stream; these are their times there):
 *   POST      a stream reached an operation and published it (a first side's
 *             ready post, an allreduce or group arrival, a persistent run's
 *             arrival);
 *   MATCH     a stream's wait for its peer's post passed (the side that
 *             copies or reduces; a persistent run's wait for the arrivals);
 *   DONE      a copy, reduce or batch published its completion (also an eager
 *             pack publishing its ready);
 *   COMPLETE  a first side's wait for that completion passed.
 * `counter` is the device address of the counter the step concerns (a
 * channel's ready or done word, a collective line), `value` its value for
 * this operation, so the steps of one message share (counter, value) pairs:
 * POST and MATCH on the first side's ready word, DONE and COMPLETE on done.
 * Recording costs one device atomic and one 32-byte store per event. */
typedef struct {
    uint64_t time_ns;     /* device wall clock, in ns */
    uint32_t kind;        /* MPIXS_TRACE_* */
    uint32_t stream;      /* device block index of the stream it happened on */
    uint64_t counter;
    uint64_t value;
} mpixs_trace_event;

#define MPIXS_TRACE_POST 1
#define MPIXS_TRACE_MATCH 2
#define MPIXS_TRACE_DONE 3
#define MPIXS_TRACE_COMPLETE 4

/* -------------------------------------------------------------- world (N ranks)
 * mpixs_world_create: make a world of nranks (1..4096) ranks on the current
 *   HIP device.  cfg may be NULL (defaults).  Allocates and clears the device
 *   tables once, here, so that no later call allocates or synchronises.
 * mpixs_world_comm: rank's handle to the world communicator (no stream
 *   attached: enqueue calls on it fail with MPIXS_ERR_COMM, as on a
 *   conventional communicator, §3.1's MPIX_STREAM_NULL semantics).
 * mpixs_world_free: MPIXS_ERR_PENDING if streams or communicators are alive.
 */
int mpixs_world_create(int nranks, const mpixs_config *cfg, mpixs_world *w);
int mpixs_world_comm(mpixs_world w, int rank, mpixs_comm *comm);
int mpixs_world_free(mpixs_world *w);
/* Block until every stream attached to the world's communicators is idle,
 * or timeout_ms passes (MPIXS_ERR_TIMEOUT).  A host-side watchdog for tests. */
int mpixs_world_wait(mpixs_world w, int timeout_ms);
/* Wake every device and host wait of the world with MPIXS_ERR_ABORTED (they
 * skip their data movement).  The world is unusable afterwards. */
int mpixs_world_abort(mpixs_world w);

/* -------------------------------------------------------------------- info
 * Key/value hints (§3.2).  mpixs_info_set_hex stores vallen bytes of value as
 * lower-case hex text (two characters per byte, memory order).  A stream for
 * a HIP stream is created from an info with type="hipStream_t" and value set
 * with mpixs_info_set_hex(info, "value", &stream, sizeof(hipStream_t)), as in
 * the paper's GPU example (§6).
 */
int mpixs_info_create(mpixs_info *info);
int mpixs_info_set(mpixs_info info, const char *key, const char *value);
int mpixs_info_set_hex(mpixs_info info, const char *key, const void *value, int vallen);
int mpixs_info_get(mpixs_info info, const char *key, char *value, int valuelen, int *flag);
int mpixs_info_free(mpixs_info *info);

/* ------------------------------------------------------------------ stream
 * mpixs_stream_create (§3.1, MPIX_Stream_create): a serial execution context
 *   bound to an endpoint of the world's pool.  info NULL: a host-thread
 *   stream (no GPU stream; enqueue calls on its communicators fail).
 *   type="hipStream_t": a GPU stream, value decoded from hex.  Fails with
 *   MPIXS_ERR_NO_ENDPOINT when the pool is empty (policy 0).
 * mpixs_stream_free (§3.1, MPIX_Stream_free): may fail with
 *   MPIXS_ERR_PENDING while communicators use the stream or operations
 *   enqueued on it have not completed; the stream then stays valid.
 * mpixs_stream_get_error: the first asynchronous error of operations that
 *   ran on the stream (0 if none).  Synchronise the HIP stream first.
 */
int mpixs_stream_create(mpixs_world w, mpixs_info info, mpixs_stream *s);
int mpixs_stream_free(mpixs_stream *s);
int mpixs_stream_get_error(mpixs_stream s, int *first_error);

/* ------------------------------------------------------------ communicator
 * mpixs_comm_create_with_stream (§3.3, MPIX_Stream_comm_create): collective
 *   over the parent's ranks; every rank thread calls it with its own parent
 *   handle and stream (MPIXS_STREAM_NULL allowed per rank).  A stream
 *   attached to the parent is not inherited (§3.3).  Blocks until all
 *   ranks have called it.  Communicators match messages independently of
 *   each other (§2.1).
 * mpixs_comm_free: frees this rank's handle; MPIXS_ERR_PENDING while
 *   requests of the handle are outstanding.
 */
int mpixs_comm_create_with_stream(mpixs_comm parent, mpixs_stream s, mpixs_comm *newcomm);
int mpixs_comm_free(mpixs_comm *comm);
int mpixs_comm_rank(mpixs_comm comm, int *rank);
int mpixs_comm_size(mpixs_comm comm, int *size);

/* --------------------------------------------------------------- datatypes
 * MPI derived datatypes over one basic type (§3.4 takes MPI datatypes; §4.5
 * notes GPU collective libraries move only contiguous intrinsic types).
 * Typemap meaning is MPI's: contiguous(n, T) places copy i at i*extent(T);
 * vector(count, bl, stride, T) places element j of block i at
 * (i*stride + j)*extent(T); indexed(count, bls, displs, T) places element j
 * of block i at (displs[i] + j)*extent(T).  Counts, blocklengths, strides
 * and displacements must be >= 0.  A type must be committed before use;
 * commit compiles it into the form the copy kernels read (an irregular
 * indexed type: a table of its segments in the memory of the GPU current at
 * commit, MPIXS_ERR_NOMEM / MPIXS_ERR_GPU if that fails).
 */
int mpixs_type_contiguous(int count, mpixs_datatype oldtype, mpixs_datatype *newtype);
int mpixs_type_vector(int count, int blocklength, int stride, mpixs_datatype oldtype,
                      mpixs_datatype *newtype);
int mpixs_type_indexed(int count, const int blocklengths[], const int displacements[],
                       mpixs_datatype oldtype, mpixs_datatype *newtype);
int mpixs_type_commit(mpixs_datatype *type);
/* mpixs_type_free releases the handle (set to MPIXS_DATATYPE_NULL).  The
 * type's description -- and an irregular indexed type's segment table in
 * device memory -- stays allocated until the process ends, since operations
 * enqueued before the free and persistent batches may still read it; a
 * process can make at most 2^20 datatypes. */
int mpixs_type_free(mpixs_datatype *type);
int mpixs_type_size(mpixs_datatype type, int64_t *bytes);
int mpixs_type_get_extent(mpixs_datatype type, int64_t *lb, int64_t *extent);

/* -------------------------------------------------------- enqueue calls (§3.4)
 * All take a stream communicator whose local stream is a GPU stream
 * (else MPIXS_ERR_COMM, §3.4).  Each returns once the operation is
 * registered; the operation runs on the stream after the operations enqueued
 * before it (§3.4).  Matching (§2.1), by mpixs_config.matching:
 *  0 (default): the k-th send from rank s to rank d with tag t on a
 *    communicator matches the k-th receive of rank d from s with tag t on it
 *    (MPI's non-overtaking order without wildcards); wildcards are rejected
 *    (MPIXS_ERR_RANK / MPIXS_ERR_TAG).
 *  1: ordered queues per destination.  A send matches the earliest posted,
 *    unmatched receive of its destination that accepts its (source, tag);
 *    a receive -- source may be MPIXS_ANY_SOURCE, tag MPIXS_ANY_TAG --
 *    matches the earliest enqueued, unmatched send to it that it accepts;
 *    otherwise the operation waits in the queue.  "Earliest" is the order in
 *    which the enqueue calls reach the library, so messages of one sender
 *    never overtake each other; which of several senders a wildcard receive
 *    meets depends on the threads' timing, as in MPI.  The status reports
 *    the matched source, tag and count.  Each message takes one block of
 *    the device matching table (cfg.max_channels in total; MPIXS_ERR_NOMEM
 *    once exhausted).  Wildcards are not allowed inside groups, and the
 *    host-synchronised calls (mpixs_send / mpixs_recv) return
 *    MPIXS_ERR_COMM in this mode.
 *
 *  send_enqueue:  later work on the stream starts once buf may be reused
 *                 (the data has been copied into the matched receive buffer).
 *  recv_enqueue:  later work on the stream sees the received data; status
 *                 (may be NULL) is written on the stream.
 *  isend/irecv_enqueue: later work may start before the transfer; *req
 *                 completes with wait_enqueue / waitall_enqueue.
 *  wait_enqueue:  later work on the stream starts after the request's
 *                 transfer; *req is consumed and set to NULL at this call.
 *  waitall_enqueue: requests must all belong to one stream (§3.4), else
 *                 MPIXS_ERR_STREAM; statuses may be NULL.
 *  Buffers (§6's GPU example; ownership stays with the caller): the bytes a
 *  message or allreduce touches must lie in device memory (hipMalloc,
 *  managed memory, torch tensors on the device) and, where HIP knows the
 *  allocation's range, inside that allocation; a status (or a waitall
 *  status array) may also lie in pinned host memory (hipHostMalloc).
 *  Anything else -- pageable host memory above all -- is MPIXS_ERR_BUFFER at
 *  the call, with no side effect, checked after the other arguments and the
 *  size limit below, with
 *  hipPointerGetAttributes / hipMemGetAddressRange.  Each stream keeps the
 *  ranges it has found valid (16 allocations, replaced round-robin), so a
 *  range freed and reused for other memory while the stream lives still
 *  passes as the allocation it was.  Zero-byte messages are not checked.
 *  Sizes: a message whose datatype is dense (its element is one contiguous
 *  block: a basic type, a contiguous type, a vector or indexed type that
 *  reduces to one block) may have any byte count; any other message must
 *  stay below 2^32 bytes (else MPIXS_ERR_COUNT, with no side effect).
 *
 * Host blocking: a call never waits for the GPU.  A call whose stream must
 * wait for the peer's stream may wait, on the host, until the peer thread
 * has *enqueued* its matching operation (blocking send/recv, wait of a
 * request whose peer has not arrived yet, allreduce of a rank that is not
 * the last to arrive), so that a device wait is never queued ahead of what
 * it waits for.  That host wait gives up after cfg.timeout_ms with
 * MPIXS_ERR_TIMEOUT.
 */
int mpixs_send_enqueue(const void *buf, int count, mpixs_datatype datatype, int dest, int tag,
                       mpixs_comm comm);
int mpixs_recv_enqueue(void *buf, int count, mpixs_datatype datatype, int source, int tag,
                       mpixs_comm comm, mpixs_status *status);
int mpixs_isend_enqueue(const void *buf, int count, mpixs_datatype datatype, int dest, int tag,
                        mpixs_comm comm, mpixs_request *request);
int mpixs_irecv_enqueue(void *buf, int count, mpixs_datatype datatype, int source, int tag,
                        mpixs_comm comm, mpixs_request *request);
int mpixs_wait_enqueue(mpixs_request *request, mpixs_status *status);
int mpixs_waitall_enqueue(int count, mpixs_request requests[], mpixs_status statuses[]);

/* allreduce_enqueue (§3.4 extends enqueue to collectives): MPI_Allreduce on
 * a contiguous basic type (int32, int64, float32, float64) with SUM, PROD,
 * MIN or MAX.  Every rank of the communicator calls it; the k-th call of
 * each rank forms one instance.  The result is, element by element, the
 * left fold over ranks 0..N-1 in that order (so float results are
 * reproducible).  sendbuf may be MPIXS_IN_PLACE (input taken from recvbuf).
 * At most 64 ranks per communicator. */
int mpixs_allreduce_enqueue(const void *sendbuf, void *recvbuf, int count,
                            mpixs_datatype datatype, mpixs_op op, mpixs_comm comm);

/* ---------------------------------------------------------------- batching
 * Groups fuse many enqueued messages into one kernel.  The paper's enqueue
 * semantics (§3.4) let an implementation move a nonblocking message at any
 * point between its call and its wait; a group widens that window to the
 * whole group: between mpixs_group_start(comm) and mpixs_group_end(comm) a
 * rank's send / recv / isend / irecv / wait / waitall_enqueue calls on comm
 * are recorded instead of enqueued (argument errors are still returned at
 * once), and mpixs_group_end enqueues them all.
 *
 *  mpixs_group_end is collective over comm (every rank calls it, possibly
 *  with an empty group; at most 64 ranks).  The rank that arrives last
 *  matches the grouped operations of all ranks (the i-th grouped send of s
 *  to d with tag t matches the i-th grouped receive of d from s with tag t)
 *  and enqueues on its own stream one wait for all ranks' streams to reach
 *  their group_end, one batch kernel that performs every copy of the group
 *  (tiles of up to 1024 units scheduled over the whole grid) and writes the
 *  receive statuses, and a completion signal; every other rank's stream
 *  waits for that signal.  So later work on any rank's stream starts after
 *  all copies of the group.  Blocking calls inside a group complete at
 *  group_end; requests created inside a group complete at group_end too
 *  (waiting on them inside or after the group only delivers the status).
 *  Every grouped send must be matched inside the same group instance, else
 *  group_end returns MPIXS_ERR_ARG on every rank and no copy of the group
 *  runs.  A channel used inside groups must not also be used outside them.
 *  allreduce_enqueue inside a group is recorded too: the i-th grouped
 *  allreduce of every rank forms the group's i-th reduction, which the
 *  launching rank's stream runs after the batch kernel, in order (so a
 *  group of many small allreduces costs one arrival and one wait per rank
 *  plus the reduce kernels, instead of two launches per rank each).
 *  When the group's allreduces all have one datatype and operation, each
 *  reads at most 64 MiB over all ranks, and no byte of any of their buffers
 *  belongs to two of them, they run as one reduce kernel (their order
 *  cannot change a result then); stats.reductions_merged counts them.
 *  Ranks that grouped different numbers of allreduces, or whose i-th calls
 *  differ in count, datatype or operation, make group_end (or
 *  group_end_init) return MPIXS_ERR_ARG on every rank; nothing of the group
 *  runs.  Reductions must not read or write buffers that the group's
 *  messages write.
 *  mpixs_group_end waits on the host until every rank has called it.
 */
/* --------------------------------------- multiplex stream communicators (§3.5)
 * mpixs_comm_create_multiplex (the paper's MPIX_Stream_comm_create_multiple):
 *   collective over parent; every rank attaches `count` (0..64) of its GPU
 *   streams, which become its stream indices 0..count-1 (an index is a rank
 *   for threads).  Errors: MPIXS_ERR_STREAM for a NULL or non-GPU stream or
 *   one of another world, MPIXS_ERR_ARG for a bad count.  The ordinary
 *   enqueue calls and allreduce fail on such a communicator with
 *   MPIXS_ERR_COMM (it has no single local stream).
 * mpixs_stream_{send,recv,isend,irecv}_enqueue (the paper's MPIX_Stream_send
 *   family, enqueued): the operation is enqueued on the local stream of the
 *   local index (src_idx for a send, dst_idx for a receive) and addresses
 *   the remote stream of the other index; a receive may use
 *   MPIXS_ANY_SOURCE, MPIXS_ANY_TAG and MPIXS_ANY_INDEX (src_idx).  Matching
 *   is ordered-queue matching per destination endpoint (rank, stream index)
 *   -- the rule documented for mpixs_config.matching = 1, whatever that
 *   setting -- and the status reports the sender's rank, stream index
 *   (source_index), tag and count.  Semantics of completion, requests and
 *   host blocking are those of the enqueue calls above; requests belong to
 *   the stream they were enqueued on (waitall across streams:
 *   MPIXS_ERR_STREAM).  Argument errors: MPIXS_ERR_RANK for a peer or index
 *   out of range, MPIXS_ERR_TAG, MPIXS_ERR_COUNT, MPIXS_ERR_TYPE,
 *   MPIXS_ERR_BUFFER, MPIXS_ERR_COMM on a communicator that is not
 *   multiplex; an erroneous call has no side effect. */
int mpixs_comm_create_multiplex(mpixs_comm parent, int count, const mpixs_stream streams[],
                                mpixs_comm *comm);
int mpixs_stream_send_enqueue(const void *buf, int count, mpixs_datatype datatype, int dest,
                              int tag, mpixs_comm comm, int src_idx, int dst_idx);
int mpixs_stream_recv_enqueue(void *buf, int count, mpixs_datatype datatype, int source, int tag,
                              mpixs_comm comm, int src_idx, int dst_idx, mpixs_status *status);
int mpixs_stream_isend_enqueue(const void *buf, int count, mpixs_datatype datatype, int dest,
                               int tag, mpixs_comm comm, int src_idx, int dst_idx,
                               mpixs_request *request);
int mpixs_stream_irecv_enqueue(void *buf, int count, mpixs_datatype datatype, int source, int tag,
                               mpixs_comm comm, int src_idx, int dst_idx, mpixs_request *request);

int mpixs_group_start(mpixs_comm comm);
int mpixs_group_end(mpixs_comm comm);

/* ----------------------------------------------------- persistent batches
 * A group that is run many times (a halo exchange or a batch of messages
 * repeated every step) need not be matched and planned every time.  The
 * model is MPI's persistent requests (init once, start many times) applied
 * to an enqueued group:
 *
 *  mpixs_group_end_init(comm, &batch) ends the rank's current group like
 *   mpixs_group_end -- collective, every rank of comm calls it for the same
 *   group instance -- but moves no data and enqueues nothing.  The last rank
 *   to arrive matches and plans the group once into device memory (one
 *   descriptor per message, a tile schedule, and counters of its own);
 *   every rank receives its handle in *batch (NULL on error).  Errors, the
 *   same on every rank: MPIXS_ERR_ARG if a grouped send or receive is
 *   unmatched, if a request created in the group is not waited for inside
 *   it, or if some ranks ended the instance with mpixs_group_end instead;
 *   MPIXS_ERR_NOMEM / MPIXS_ERR_GPU if the plan cannot be stored.  The
 *   buffers, datatypes and statuses named by the group's calls must stay
 *   valid until the batch is freed.
 *  mpixs_batch_start_enqueue(batch) enqueues one run of the whole group on
 *   the rank's stream: each run moves every message of the group again, from
 *   the send buffers' contents when the run executes, and writes the
 *   receive statuses.  Every rank starts its handle the same number of
 *   times; run k of all ranks is one instance, and later work on any rank's
 *   stream starts after all copies of that run.  One rank (the one that
 *   planned it) launches a wait for the others' arrival, one batch kernel
 *   and a signal; every other rank enqueues an arrival and a wait.  The
 *   kernels keep their counters relative (they count runs on the device),
 *   so their arguments are the same for every run and the launching rank's
 *   part can be replayed as one HIP graph (mpixs_config.batch_graph).  With
 *   mpixs_config.batch_sync = 1 the arrivals and the completion are HIP
 *   events instead (each other rank records one, the launching rank's
 *   stream waits for them, runs the batch kernel and records one that the
 *   other streams wait for): no arrival, wait or signal kernel.  Like
 *   the other enqueue calls it may wait on the host until the peers have
 *   enqueued their part of the run, never for GPU work.
 *   MPIXS_ERR_REQUEST for a NULL handle; MPIXS_ERR_ARG inside an open group.
 *  mpixs_batch_free(&batch): per rank; the last rank to free it waits for
 *   the device to finish and releases the plan.  Handles keep their
 *   communicator busy (mpixs_comm_free fails with MPIXS_ERR_PENDING).
 */
int mpixs_group_end_init(mpixs_comm comm, mpixs_batch *batch);
int mpixs_batch_start_enqueue(mpixs_batch batch);
int mpixs_batch_free(mpixs_batch *batch);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * mpixs_group_end_init_static(comm, &batch) is mpixs_group_end_init whose
 * plan (counters, descriptors, tile schedule) goes into a static region of
 * 4 MiB (4,194,304 bytes) that each GPU holds for the life of the process,
 * instead of memory allocated for it; it calls no hipMalloc or hipFree and
 * creates no graph or event (runs use the device counters whatever
 * mpixs_config.batch_graph and batch_sync say).  The plan needs 128 bytes
 * per rank and 128 more, 224 per message, 8 per batch-kernel workgroup and,
 * for merged allreduces, 24 per allreduce and 16 per allreduce and rank,
 * each part rounded up to 256 bytes; a larger one fails with
 * MPIXS_ERR_NOMEM on every rank, nothing planned.  One region per GPU: the
 * region holds the last such plan made on the GPU, and a start of an earlier
 * one returns MPIXS_ERR_REQUEST.  Making a new one while runs of the
 * previous one are still executing on the GPU is a race (the caller orders
 * them); counters start at zero with every plan.  Collective over comm, all
 * ranks calling this same function (else MPIXS_ERR_ARG on every rank);
 * start and free it like any batch. */
int mpixs_group_end_init_static(mpixs_comm comm, mpixs_batch *batch);

/* ------------------------------------ conventional, host-synchronised calls
 * The comparison path of §2.4: MPI calls that run in the CPU context and
 * fully synchronise with the GPU.  Each call synchronises its rank's HIP
 * stream, matches on the host, launches one copy (or reduce) kernel -- the
 * same kernels as the enqueue path -- and synchronises again before it
 * returns.  They take stream communicators (they need the HIP stream) and
 * match only among themselves: mixing them with enqueue calls on one
 * channel is not supported.
 */
int mpixs_send(const void *buf, int count, mpixs_datatype datatype, int dest, int tag,
               mpixs_comm comm);
int mpixs_recv(void *buf, int count, mpixs_datatype datatype, int source, int tag,
               mpixs_comm comm, mpixs_status *status);
int mpixs_allreduce(const void *sendbuf, void *recvbuf, int count, mpixs_datatype datatype,
                    mpixs_op op, mpixs_comm comm);

/* ------------------------------------------------------------- diagnostics */
typedef struct {
    uint64_t kernels_post;      /* one-thread "stream reached this point" kernels */
    uint64_t kernels_wait;      /* one-wave wait kernels */
    uint64_t kernels_copy;      /* copy kernels (fused or not) */
    uint64_t kernels_reduce;    /* reduce kernels */
    uint64_t bytes_copied;      /* payload bytes moved by copy kernels */
    uint64_t bytes_reduced;     /* bytes read + written by reduce kernels */
    uint64_t host_waits;        /* enqueue calls that waited for a peer's enqueue */
    uint64_t timed_copy;        /* profile=1: copy kernels timed with HIP events */
    double copy_ms;             /* profile=1: sum of their event durations */
    uint64_t timed_reduce;
    double reduce_ms;
    uint64_t host_sleeps;       /* host waits that went to sleep (futex) at least once */
    uint64_t host_sleep_timeouts; /* sleeps that ended by their 1 ms bound, not a wake-up */
    uint64_t groups_planned;    /* group instances matched and planned (one-shot or init) */
    double plan_ms;             /* host time the planning ranks spent on them */
    uint64_t reductions_merged; /* grouped allreduces run inside one merged reduce kernel */
    uint64_t channels_recycled; /* matching-table blocks handed to a new channel (§3.1 frees) */
    uint64_t streams_recycled;  /* stream blocks of freed streams taken by new streams */
    uint64_t comm_lines_recycled; /* collective lines of freed communicators reused */
    uint64_t eager_sends;       /* blocking sends complete on the sender's stream before
                                   their receive was enqueued (eager; empty ones included) */
} mpixs_stats;

/* Counters of the world since creation (or the last reset).  With
 * cfg.profile = 1 the event durations are collected here, which requires
 * the streams to be idle (call after synchronising). */
int mpixs_world_get_stats(mpixs_world w, mpixs_stats *stats);
int mpixs_world_reset_stats(mpixs_world w);
/* Copy the newest min(max, kept) recorded trace events, oldest first, into
 * events[0 ..]; *copied receives how many were copied and *total the number
 * recorded since the world was created, of which the ring keeps the last
 * trace_events (rounded up to a power of two).  Call while the world's
 * streams are idle (the copy does not order itself after their kernels).
 * MPIXS_ERR_ARG when tracing is off, for a NULL copied or total, or a
 * negative max (events may be NULL when max is 0). */
int mpixs_world_trace(mpixs_world w, mpixs_trace_event *events, int64_t max, int64_t *copied,
                      int64_t *total);
const char *mpixs_error_string(int err);

#ifdef __cplusplus
}
#endif
#endif /* MPIXS_H */
