/*
 * mpixs_driver.h -- native multi-threaded program runner for libmpixs.
 *
 * Ranks of a world are host threads (one per stream).  This runner starts
 * one C++ thread per entry of `threads`, releases them together, and has
 * each issue its op list through the public libmpixs calls -- the enqueue
 * calls or, in host-synchronised mode, the conventional ones -- so that
 * benchmarks measure the library and not an interpreter.  It is a harness:
 * every operation it performs goes through include/mpixs.h.
 */
#ifndef MPIXS_DRIVER_H
#define MPIXS_DRIVER_H

#include <stdint.h>

#include "mpixs.h"

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MPIXS_DRV_SEND = 1,      /* send_enqueue (host-synced mode: mpixs_send)        */
    MPIXS_DRV_ISEND = 2,     /* isend_enqueue into request slot `req`              */
    MPIXS_DRV_RECV = 3,      /* recv_enqueue (host-synced mode: mpixs_recv)        */
    MPIXS_DRV_IRECV = 4,     /* irecv_enqueue into request slot `req`              */
    MPIXS_DRV_WAITALL = 5,   /* waitall_enqueue over slots [req, req + nreq);
                                statuses at `status` (array) or none               */
    MPIXS_DRV_ALLREDUCE = 6, /* allreduce_enqueue(buf, buf2, ...) (host-synced:
                                mpixs_allreduce); buf == 1 means in place          */
    MPIXS_DRV_MARK = 7,      /* record HIP event number `req` of this thread       */
    MPIXS_DRV_GROUP_START = 8, /* mpixs_group_start(comm)                          */
    MPIXS_DRV_GROUP_END = 9,   /* mpixs_group_end(comm)                            */
    MPIXS_DRV_GROUP_INIT = 10, /* mpixs_group_end_init(comm, &batches[req])        */
    MPIXS_DRV_BATCH_START = 11, /* mpixs_batch_start_enqueue(batches[req])         */
    MPIXS_DRV_BATCH_FREE = 12, /* mpixs_batch_free(&batches[req])                  */
    /* multiplex communicators: src_idx in `op`, dst_idx in `pad` */
    MPIXS_DRV_STREAM_SEND = 13,  /* mpixs_stream_send_enqueue                      */
    MPIXS_DRV_STREAM_ISEND = 14, /* mpixs_stream_isend_enqueue into slot `req`     */
    MPIXS_DRV_STREAM_RECV = 15,  /* mpixs_stream_recv_enqueue                      */
    MPIXS_DRV_STREAM_IRECV = 16, /* mpixs_stream_irecv_enqueue into slot `req`     */
    MPIXS_DRV_GROUP_INIT_STATIC = 17 /* mpixs_group_end_init_static(comm, &batches[req]) */
};

typedef struct {
    int32_t kind;
    int32_t comm;      /* index into this thread's communicator list */
    int32_t peer;
    int32_t tag;
    int32_t count;
    int32_t datatype;
    int32_t op;
    int32_t req;
    int32_t nreq;
    int32_t pad;
    uint64_t buf;      /* device address */
    uint64_t buf2;     /* allreduce receive buffer */
    uint64_t status;   /* device address of an mpixs_status (array for waitall), or 0 */
} mpixs_drv_op;

typedef struct {
    mpixs_comm comms[16];    /* this thread's communicators */
    int32_t ncomms;
    int32_t nmarks;          /* HIP events this thread may record (MPIXS_DRV_MARK) */
    void *hip_stream;        /* the thread's hipStream_t, synchronised at the end */
    const mpixs_drv_op *ops;
    int64_t nops;
    int32_t max_reqs;        /* request slots */
    int32_t nbatches;        /* persistent batch slots at `batches` */
    mpixs_batch *batches;    /* caller-owned, so batches outlive one run */
} mpixs_drv_thread;

typedef struct {
    double seconds;          /* max over threads of (end - common start), end taken after
                                the thread's stream has drained */
    int32_t first_error;     /* first non-zero return code, 0 if none */
    int32_t error_thread;
    int64_t error_op;
    double enqueue_seconds;  /* max over threads of (return of its last call - common start),
                                before its stream is synchronised: the host's share */
} mpixs_drv_result;

/* ------------------------------------------------------------- serving
 * An open-loop request server over the enqueue path.  Requests arrive at
 * given times; a scheduler thread admits them first come, first served, each
 * once it has arrived and its buffers fit in a device arena of
 * `budget_bytes` (waiting for earlier requests to finish if they do not),
 * after which every participant's rank thread enqueues its part on its
 * stream: the sender fills its buffer with the request's payload and sends
 * (send_enqueue, or isend_enqueue + wait_enqueue), the receiver receives and
 * a checksum of the received bytes is written to host memory; for an
 * allreduce every rank fills its input, calls allreduce_enqueue (int32 SUM
 * over all ranks) and checksums its own output, the request's checksum being
 * the sum over ranks r of (2r + 1) times rank r's checksum (so with every
 * output equal to the fold, n^2 times its checksum, modulo 2^64).  A reaper thread
 * watches the completion flags (written by the device), frees the buffers
 * and timestamps the requests, so later arrivals are admitted as memory
 * frees up while earlier requests are still on the GPU.
 *
 * Payload byte j of a buffer with seed s is byte (j mod 8) of
 * splitmix64(s * 2^32 + floor(j / 8)) (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014); the checksum of n bytes is
 * the sum over j of byte_j * (j + 1) modulo 2^64.  An allreduce rank r uses
 * seed s + r. */
enum { MPIXS_DRV_REQ_SENDRECV = 0, MPIXS_DRV_REQ_ISEND_WAIT = 1, MPIXS_DRV_REQ_ALLREDUCE = 2 };

typedef struct {
    int32_t kind;
    int32_t src;         /* point-to-point: sender */
    int32_t dst;         /* point-to-point: receiver */
    int32_t pad;
    int64_t bytes;       /* message bytes; allreduce: bytes per rank (multiple of 4) */
    double arrival_us;   /* arrival time after the start */
    uint64_t seed;
} mpixs_drv_req;

typedef struct {
    double admit_us;     /* when the scheduler admitted it (after the start) */
    double done_us;      /* when the reaper saw its completion flag */
    uint64_t checksum;   /* device checksum of the received / reduced bytes */
    int32_t error;       /* first error of an enqueue call of the request */
    int32_t pad;
} mpixs_drv_req_result;

/* Serve nreq requests (sorted by arrival) with one thread per rank of the
 * communicators comms[0..nranks-1] (each with its GPU stream in streams[]).
 * Admission in arrival order keeps the admitted requests a prefix of the
 * schedule, so a request never waits for memory held by requests that
 * depend on it.
 * Point-to-point requests need src != dst (a synchronous send to oneself on
 * one stream cannot complete).  Returns MPIXS_ERR_ARG (nothing run) for an
 * unsorted list, an unknown kind, out-of-range ranks or sizes, or an
 * allreduce size that is not a multiple of 4; MPIXS_ERR_NOMEM if the budget
 * cannot be allocated or a request does not fit it; otherwise the first
 * error of an enqueue call (0 if none).  *wall_s receives the time from the
 * start to the last completion.  The buffers live in one device allocation
 * of budget_bytes made by this call and freed before it returns.
 * Capture: for k < ncapture, request capture[2k] also copies its result
 * bytes, before they are checksummed, to capture_dev + capture[2k+1] (device
 * memory of the caller): the received bytes, or for an allreduce every
 * rank's output, rank r's at offset r * bytes.  capture may be NULL when
 * ncapture is 0.
 * flags: MPIXS_DRV_SERVE_HOST_SYNCED serves with the host-synchronised calls
 * (mpixs_send / mpixs_recv for both point-to-point kinds, mpixs_allreduce),
 * the comparison path of §2.4 with the same schedule, buffers and checksums,
 * instead of the enqueue calls (send/recv_enqueue, isend_enqueue +
 * wait_enqueue, allreduce_enqueue); MPIXS_DRV_SERVE_RANK0_SUM checksums an
 * allreduce's output on rank 0 only (its checksum is then the fold's
 * checksum) instead of on every rank.  Other bits: MPIXS_ERR_ARG. */
#define MPIXS_DRV_SERVE_HOST_SYNCED 1
#define MPIXS_DRV_SERVE_RANK0_SUM 2
int mpixs_drv_serve(mpixs_world world, int nranks, const mpixs_comm *comms,
                    void *const *streams, const mpixs_drv_req *reqs, int64_t nreq,
                    int64_t budget_bytes, mpixs_drv_req_result *results, double *wall_s,
                    const int64_t *capture, int64_t ncapture, void *capture_dev, int flags);

/* ------------------------------------------------ host message-rate model
 * A CPU-only analog of the paper's multithreaded message-rate measurement
 * (§5.3, Fig. 3).  Thread i of a simulated sender process sends
 * msgs_per_pair 8-byte messages to thread i of a simulated receiver process
 * (npairs pairs, 2 * npairs threads), each thread on its own context, in
 * windows of `window` isends (irecvs) closed by a waitall; at most two
 * windows are in flight.  The message engine (request objects, posted and
 * unexpected queues, progress) is synchronised by policy 0 (one critical
 * section per process, held for each call and yielded between progress
 * passes), 1 (one mutex per context, taken separately on the send path, the
 * receive path, each progress pass and each request release) or 2 (stream
 * contexts: no locks).  Completion flags and request reference counts are
 * atomic in every policy.  *msgs_per_s receives the total message rate;
 * *checksum (may be NULL) the sum over pairs i and messages n of
 * (i * 2^40 + n) * (n + 1) modulo 2^64 as received, which holds only if
 * every message arrived once and in order.  Returns 0, or 1 for bad
 * arguments (npairs 1..256, policy 0..2, msgs_per_pair >= 1, window
 * 1..1024).  Does not touch the GPU. */
int mpixs_drv_host_msgrate(int npairs, int policy, int64_t msgs_per_pair, int window,
                           double *msgs_per_s, uint64_t *checksum);

/* Run the threads; mode 0 = enqueue calls, 1 = host-synchronised calls.
 * marks_ms (optional, nthreads * max nmarks doubles, row-major by thread)
 * receives the time of every recorded mark relative to thread 0's mark 0.
 * On an error the world is aborted so that every thread returns. */
int mpixs_drv_run(mpixs_world world, int nthreads, const mpixs_drv_thread *threads, int mode,
                  mpixs_drv_result *result, double *marks_ms);

#ifdef __cplusplus
}
#endif
#endif
