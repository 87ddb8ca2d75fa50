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
    MPIXS_DRV_GROUP_END = 9    /* mpixs_group_end(comm)                            */
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
    mpixs_comm comms[8];     /* this thread's communicators */
    int32_t ncomms;
    int32_t nmarks;          /* HIP events this thread may record (MPIXS_DRV_MARK) */
    void *hip_stream;        /* the thread's hipStream_t, synchronised at the end */
    const mpixs_drv_op *ops;
    int64_t nops;
    int32_t max_reqs;        /* request slots */
    int32_t pad;
} mpixs_drv_thread;

typedef struct {
    double seconds;          /* max over threads of (end - common start), end taken after
                                the thread's stream has drained */
    int32_t first_error;     /* first non-zero return code, 0 if none */
    int32_t error_thread;
    int64_t error_op;
} mpixs_drv_result;

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
