/*
 * mpixs_debug.h -- host-side introspection of libmpixs for tests.
 *
 * Not part of the enqueue interface: plan introspection (no GPU work) and
 * kernel timing for benchmarks.
 */
#ifndef MPIXS_DEBUG_H
#define MPIXS_DEBUG_H

#include <stdint.h>

#include "mpixs.h"

#ifdef __cplusplus
extern "C" {
#endif

/* The copy plan the library would launch for a matched message of nbytes
 * packed bytes sent as (sbuf, scount, stype) and received into (rbuf,
 * rcount, rtype): *unit_bytes receives the unit size of the copy kernel,
 * *nunits the number of units, and for the first min(nunits, max_units)
 * units src_addr[u] / dst_addr[u] receive the byte addresses unit u is read
 * from and written to (either array may be NULL).  sbuf and rbuf are only
 * used as numbers.  Datatypes need not be committed.  Errors:
 * MPIXS_ERR_TYPE for an unknown datatype, MPIXS_ERR_ARG for NULL outputs. */
int mpixs_debug_copy_plan(uint64_t sbuf, int scount, mpixs_datatype stype, uint64_t rbuf,
                          int rcount, mpixs_datatype rtype, int64_t nbytes, int64_t max_units,
                          uint64_t *src_addr, uint64_t *dst_addr, int *unit_bytes,
                          int64_t *nunits);

/* Time the copy kernel of one message at its real shape: plan the copy of
 * (sbuf, scount, stype) into (rbuf, rcount, rtype) as the enqueue path
 * would for a large message, launch its data kernel `reps` times back to
 * back on the HIP stream `hip_stream` between one pair of HIP events, wait
 * for the stream, and store the average per launch in *avg_us (and the unit
 * size in *unit_bytes if not NULL).  Buffers must be device memory, types
 * committed.  This call allocates a small scratch block and synchronises
 * the stream; it is for benchmarks, not for the enqueue path. */
int mpixs_debug_time_copy(void *hip_stream, const void *sbuf, int scount, mpixs_datatype stype,
                          void *rbuf, int rcount, mpixs_datatype rtype, int reps, double *avg_us,
                          int *unit_bytes);

/* Time the batch kernel of a persistent batch at its real shape: launch it
 * `reps` times back to back (after one untimed launch) on the HIP stream
 * `hip_stream` between one pair of HIP events, without the waits and the
 * signal of a run, wait for the stream, and store the average per launch in
 * *avg_us, the group's payload bytes (sum over its messages) in
 * *payload_bytes and the launch's workgroups in *workgroups (either may be
 * NULL).  Each launch performs every copy of the group again, so the
 * buffers hold the same bytes afterwards.  No run of the batch may be in
 * flight.  MPIXS_ERR_REQUEST for a NULL handle, MPIXS_ERR_ARG for reps < 1
 * or avg_us NULL. */
int mpixs_debug_time_batch(mpixs_batch batch, void *hip_stream, int reps, double *avg_us,
                           int64_t *payload_bytes, int *workgroups);

#ifdef __cplusplus
}
#endif
#endif
