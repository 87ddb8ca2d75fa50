"""Thin ctypes binding of libmpixs.so.

Every function here has the name of the C entry point it calls and only
marshals arguments: Python ints or objects with ``data_ptr()`` (torch
tensors) become pointers, output handles come back as the second element of
a returned tuple, and every call returns the library's error code first.
No computation of the method happens in Python; if the shared library is
missing the import of this module fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpixs.so")

# ---------------------------------------------------------------- constants
SUCCESS = 0
ERR_NAMES = {
    0: "SUCCESS", 1: "ERR_ARG", 2: "ERR_COUNT", 3: "ERR_TYPE", 4: "ERR_RANK", 5: "ERR_TAG",
    6: "ERR_COMM", 7: "ERR_STREAM", 8: "ERR_REQUEST", 9: "ERR_BUFFER", 10: "ERR_NO_ENDPOINT",
    11: "ERR_PENDING", 12: "ERR_NOMEM", 13: "ERR_OP", 14: "ERR_TRUNCATE", 15: "ERR_TIMEOUT",
    16: "ERR_ABORTED", 17: "ERR_GPU", 18: "ERR_INTERN",
}
ANY_SOURCE = -2
ANY_TAG = -1
ANY_INDEX = -3
IN_PLACE = 1

UINT8, INT8, INT32, FLOAT32, INT64, FLOAT64 = 1, 2, 3, 4, 5, 6
BASIC = {"uint8": UINT8, "int8": INT8, "int32": INT32, "float32": FLOAT32,
         "int64": INT64, "float64": FLOAT64}
SUM, PROD, MIN, MAX = 1, 2, 3, 4
OPS = {"sum": SUM, "prod": PROD, "min": MIN, "max": MAX}


class Config(ctypes.Structure):
    _fields_ = [("max_streams", ctypes.c_int32), ("endpoint_policy", ctypes.c_int32),
                ("fuse_max_bytes", ctypes.c_int32), ("timeout_ms", ctypes.c_int32),
                ("max_channels", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("max_collectives", ctypes.c_int32), ("batch_arena_mib", ctypes.c_int32),
                ("batch_tile", ctypes.c_int32), ("batch_max_wg", ctypes.c_int32),
                ("batch_graph", ctypes.c_int32), ("batch_nontemporal", ctypes.c_int32),
                ("matching", ctypes.c_int32), ("batch_sync", ctypes.c_int32),
                ("eager_max_bytes", ctypes.c_int32), ("eager_arena_mib", ctypes.c_int32),
                ("trace_events", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class Status(ctypes.Structure):
    _fields_ = [("source", ctypes.c_int32), ("tag", ctypes.c_int32), ("error", ctypes.c_int32),
                ("source_index", ctypes.c_int32), ("count_bytes", ctypes.c_int64)]


STATUS_BYTES = ctypes.sizeof(Status)


class TraceEvent(ctypes.Structure):
    _fields_ = [("time_ns", ctypes.c_uint64), ("kind", ctypes.c_uint32),
                ("stream", ctypes.c_uint32), ("counter", ctypes.c_uint64), ("value", ctypes.c_uint64)]


TRACE_POST, TRACE_MATCH, TRACE_DONE, TRACE_COMPLETE = 1, 2, 3, 4


class Stats(ctypes.Structure):
    _fields_ = [("kernels_post", ctypes.c_uint64), ("kernels_wait", ctypes.c_uint64),
                ("kernels_copy", ctypes.c_uint64), ("kernels_reduce", ctypes.c_uint64),
                ("bytes_copied", ctypes.c_uint64), ("bytes_reduced", ctypes.c_uint64),
                ("host_waits", ctypes.c_uint64), ("timed_copy", ctypes.c_uint64),
                ("copy_ms", ctypes.c_double), ("timed_reduce", ctypes.c_uint64),
                ("reduce_ms", ctypes.c_double), ("host_sleeps", ctypes.c_uint64),
                ("host_sleep_timeouts", ctypes.c_uint64), ("groups_planned", ctypes.c_uint64),
                ("plan_ms", ctypes.c_double), ("reductions_merged", ctypes.c_uint64),
                ("channels_recycled", ctypes.c_uint64), ("streams_recycled", ctypes.c_uint64),
                ("comm_lines_recycled", ctypes.c_uint64), ("eager_sends", ctypes.c_uint64)]


_vp = ctypes.c_void_p
_i = ctypes.c_int
_pp = ctypes.POINTER(ctypes.c_void_p)

# name -> (argtypes)
SIGNATURES = {
    "mpixs_world_create": [_i, ctypes.POINTER(Config), _pp],
    "mpixs_world_comm": [_vp, _i, _pp],
    "mpixs_world_free": [_pp],
    "mpixs_world_wait": [_vp, _i],
    "mpixs_world_abort": [_vp],
    "mpixs_info_create": [_pp],
    "mpixs_info_set": [_vp, ctypes.c_char_p, ctypes.c_char_p],
    "mpixs_info_set_hex": [_vp, ctypes.c_char_p, _vp, _i],
    "mpixs_info_get": [_vp, ctypes.c_char_p, ctypes.c_char_p, _i, ctypes.POINTER(_i)],
    "mpixs_info_free": [_pp],
    "mpixs_stream_create": [_vp, _vp, _pp],
    "mpixs_stream_free": [_pp],
    "mpixs_stream_get_error": [_vp, ctypes.POINTER(_i)],
    "mpixs_comm_create_with_stream": [_vp, _vp, _pp],
    "mpixs_comm_free": [_pp],
    "mpixs_comm_rank": [_vp, ctypes.POINTER(_i)],
    "mpixs_comm_size": [_vp, ctypes.POINTER(_i)],
    "mpixs_type_contiguous": [_i, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "mpixs_type_vector": [_i, _i, _i, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "mpixs_type_indexed": [_i, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.c_int32,
                           ctypes.POINTER(ctypes.c_int32)],
    "mpixs_type_commit": [ctypes.POINTER(ctypes.c_int32)],
    "mpixs_type_free": [ctypes.POINTER(ctypes.c_int32)],
    "mpixs_type_size": [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)],
    "mpixs_type_get_extent": [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64)],
    "mpixs_send_enqueue": [_vp, _i, ctypes.c_int32, _i, _i, _vp],
    "mpixs_recv_enqueue": [_vp, _i, ctypes.c_int32, _i, _i, _vp, _vp],
    "mpixs_isend_enqueue": [_vp, _i, ctypes.c_int32, _i, _i, _vp, _pp],
    "mpixs_irecv_enqueue": [_vp, _i, ctypes.c_int32, _i, _i, _vp, _pp],
    "mpixs_wait_enqueue": [_pp, _vp],
    "mpixs_waitall_enqueue": [_i, _pp, _vp],
    "mpixs_allreduce_enqueue": [_vp, _vp, _i, ctypes.c_int32, ctypes.c_int32, _vp],
    "mpixs_group_start": [_vp],
    "mpixs_group_end": [_vp],
    "mpixs_group_end_init": [_vp, _pp],
    "mpixs_group_end_init_static": [_vp, _pp],
    "mpixs_comm_create_multiplex": [_vp, _i, _pp, _pp],
    "mpixs_stream_send_enqueue": [_vp, _i, ctypes.c_int32, _i, _i, _vp, _i, _i],
    "mpixs_stream_recv_enqueue": [_vp, _i, ctypes.c_int32, _i, _i, _vp, _i, _i, _vp],
    "mpixs_stream_isend_enqueue": [_vp, _i, ctypes.c_int32, _i, _i, _vp, _i, _i, _pp],
    "mpixs_stream_irecv_enqueue": [_vp, _i, ctypes.c_int32, _i, _i, _vp, _i, _i, _pp],
    "mpixs_batch_start_enqueue": [_vp],
    "mpixs_batch_free": [_pp],
    "mpixs_send": [_vp, _i, ctypes.c_int32, _i, _i, _vp],
    "mpixs_recv": [_vp, _i, ctypes.c_int32, _i, _i, _vp, _vp],
    "mpixs_allreduce": [_vp, _vp, _i, ctypes.c_int32, ctypes.c_int32, _vp],
    "mpixs_world_get_stats": [_vp, ctypes.POINTER(Stats)],
    "mpixs_world_reset_stats": [_vp],
    "mpixs_world_trace": [_vp, _vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                          ctypes.POINTER(ctypes.c_int64)],
    "mpixs_error_string": [_i],
}

_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """Load libmpixs.so (built in-tree by ``paper_2208_13707_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2208_13707_amd.build` (no fallback exists)")
        # torch ships its own HIP runtime; loaded first, it is the one the
        # library binds to, so buffers, streams and kernels share one runtime
        # (loaded the other way round, the process would hold two)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_char_p if name == "mpixs_error_string" else ctypes.c_int
        _lib = L
    return _lib


def ptr(x) -> int:
    """A device pointer from an int, None, or anything with data_ptr()."""
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def errname(rc: int) -> str:
    return ERR_NAMES.get(rc, f"ERR_{rc}")


# ---------------------------------------------------------------- wrappers
def mpixs_world_create(nranks: int, cfg: Optional[Config] = None):
    h = ctypes.c_void_p()
    rc = lib().mpixs_world_create(nranks, ctypes.byref(cfg) if cfg is not None else None,
                                  ctypes.byref(h))
    return rc, h.value


def mpixs_world_comm(world, rank: int):
    h = ctypes.c_void_p()
    rc = lib().mpixs_world_comm(world, rank, ctypes.byref(h))
    return rc, h.value


def mpixs_world_free(world):
    h = ctypes.c_void_p(world)
    return lib().mpixs_world_free(ctypes.byref(h))


def mpixs_world_wait(world, timeout_ms: int):
    return lib().mpixs_world_wait(world, timeout_ms)


def mpixs_world_abort(world):
    return lib().mpixs_world_abort(world)


def mpixs_info_create():
    h = ctypes.c_void_p()
    rc = lib().mpixs_info_create(ctypes.byref(h))
    return rc, h.value


def mpixs_info_set(info, key: str, value: str):
    return lib().mpixs_info_set(info, key.encode(), value.encode())


def mpixs_info_set_hex(info, key: str, value: bytes):
    buf = ctypes.create_string_buffer(value, len(value))
    return lib().mpixs_info_set_hex(info, key.encode(), ctypes.cast(buf, ctypes.c_void_p), len(value))


def mpixs_info_get(info, key: str, maxlen: int = 256):
    buf = ctypes.create_string_buffer(maxlen)
    flag = ctypes.c_int()
    rc = lib().mpixs_info_get(info, key.encode(), buf, maxlen, ctypes.byref(flag))
    return rc, (buf.value.decode() if flag.value else None)


def mpixs_info_free(info):
    h = ctypes.c_void_p(info)
    return lib().mpixs_info_free(ctypes.byref(h))


def mpixs_stream_create(world, info=None):
    h = ctypes.c_void_p()
    rc = lib().mpixs_stream_create(world, info, ctypes.byref(h))
    return rc, h.value


def mpixs_stream_free(stream):
    h = ctypes.c_void_p(stream)
    rc = lib().mpixs_stream_free(ctypes.byref(h))
    return rc


def mpixs_stream_get_error(stream):
    e = ctypes.c_int()
    rc = lib().mpixs_stream_get_error(stream, ctypes.byref(e))
    return rc, e.value


def mpixs_comm_create_with_stream(parent, stream):
    h = ctypes.c_void_p()
    rc = lib().mpixs_comm_create_with_stream(parent, stream, ctypes.byref(h))
    return rc, h.value


def mpixs_comm_free(comm):
    h = ctypes.c_void_p(comm)
    return lib().mpixs_comm_free(ctypes.byref(h))


def mpixs_comm_rank(comm):
    v = ctypes.c_int()
    rc = lib().mpixs_comm_rank(comm, ctypes.byref(v))
    return rc, v.value


def mpixs_comm_size(comm):
    v = ctypes.c_int()
    rc = lib().mpixs_comm_size(comm, ctypes.byref(v))
    return rc, v.value


def mpixs_type_contiguous(count: int, old: int):
    t = ctypes.c_int32()
    rc = lib().mpixs_type_contiguous(count, old, ctypes.byref(t))
    return rc, t.value


def mpixs_type_vector(count: int, bl: int, stride: int, old: int):
    t = ctypes.c_int32()
    rc = lib().mpixs_type_vector(count, bl, stride, old, ctypes.byref(t))
    return rc, t.value


def mpixs_type_indexed(bls, displs, old: int):
    n = len(bls)
    a = (ctypes.c_int * max(n, 1))(*bls)
    d = (ctypes.c_int * max(n, 1))(*displs)
    t = ctypes.c_int32()
    rc = lib().mpixs_type_indexed(n, a, d, old, ctypes.byref(t))
    return rc, t.value


def mpixs_type_commit(t: int):
    v = ctypes.c_int32(t)
    rc = lib().mpixs_type_commit(ctypes.byref(v))
    return rc, v.value


def mpixs_type_free(t: int):
    v = ctypes.c_int32(t)
    return lib().mpixs_type_free(ctypes.byref(v))


def mpixs_type_size(t: int):
    v = ctypes.c_int64()
    rc = lib().mpixs_type_size(t, ctypes.byref(v))
    return rc, v.value


def mpixs_type_get_extent(t: int):
    lb, ext = ctypes.c_int64(), ctypes.c_int64()
    rc = lib().mpixs_type_get_extent(t, ctypes.byref(lb), ctypes.byref(ext))
    return rc, lb.value, ext.value


def mpixs_send_enqueue(buf, count, dt, dest, tag, comm):
    return lib().mpixs_send_enqueue(ptr(buf), count, dt, dest, tag, comm)


def mpixs_recv_enqueue(buf, count, dt, source, tag, comm, status=None):
    return lib().mpixs_recv_enqueue(ptr(buf), count, dt, source, tag, comm, ptr(status))


def mpixs_isend_enqueue(buf, count, dt, dest, tag, comm):
    r = ctypes.c_void_p()
    rc = lib().mpixs_isend_enqueue(ptr(buf), count, dt, dest, tag, comm, ctypes.byref(r))
    return rc, r.value


def mpixs_irecv_enqueue(buf, count, dt, source, tag, comm):
    r = ctypes.c_void_p()
    rc = lib().mpixs_irecv_enqueue(ptr(buf), count, dt, source, tag, comm, ctypes.byref(r))
    return rc, r.value


def mpixs_wait_enqueue(request, status=None):
    r = ctypes.c_void_p(request)
    rc = lib().mpixs_wait_enqueue(ctypes.byref(r), ptr(status))
    return rc, r.value


def mpixs_waitall_enqueue(requests, statuses=None):
    n = len(requests)
    arr = (ctypes.c_void_p * max(n, 1))(*requests)
    rc = lib().mpixs_waitall_enqueue(n, arr, ptr(statuses))
    return rc, [arr[i] for i in range(n)]


def mpixs_allreduce_enqueue(sendbuf, recvbuf, count, dt, op, comm):
    return lib().mpixs_allreduce_enqueue(ptr(sendbuf), ptr(recvbuf), count, dt, op, comm)


def mpixs_group_start(comm):
    return lib().mpixs_group_start(comm)


def mpixs_group_end(comm):
    return lib().mpixs_group_end(comm)


def mpixs_comm_create_multiplex(parent, streams):
    """Returns (rc, communicator or None)."""
    arr = (ctypes.c_void_p * max(len(streams), 1))(*streams)
    h = ctypes.c_void_p()
    rc = lib().mpixs_comm_create_multiplex(parent, len(streams), arr, ctypes.byref(h))
    return rc, h.value


def mpixs_stream_send_enqueue(buf, count, dt, dest, tag, comm, src_idx, dst_idx):
    return lib().mpixs_stream_send_enqueue(ptr(buf), count, dt, dest, tag, comm, src_idx, dst_idx)


def mpixs_stream_recv_enqueue(buf, count, dt, source, tag, comm, src_idx, dst_idx, status=None):
    return lib().mpixs_stream_recv_enqueue(ptr(buf), count, dt, source, tag, comm, src_idx,
                                           dst_idx, ptr(status))


def mpixs_stream_isend_enqueue(buf, count, dt, dest, tag, comm, src_idx, dst_idx):
    h = ctypes.c_void_p()
    rc = lib().mpixs_stream_isend_enqueue(ptr(buf), count, dt, dest, tag, comm, src_idx, dst_idx,
                                          ctypes.byref(h))
    return rc, h.value


def mpixs_stream_irecv_enqueue(buf, count, dt, source, tag, comm, src_idx, dst_idx):
    h = ctypes.c_void_p()
    rc = lib().mpixs_stream_irecv_enqueue(ptr(buf), count, dt, source, tag, comm, src_idx,
                                          dst_idx, ctypes.byref(h))
    return rc, h.value


def mpixs_group_end_init(comm):
    """Returns (rc, batch handle or None)."""
    h = ctypes.c_void_p()
    rc = lib().mpixs_group_end_init(comm, ctypes.byref(h))
    return rc, h.value


def mpixs_group_end_init_static(comm):
    """Returns (rc, batch handle or None)."""
    h = ctypes.c_void_p()
    rc = lib().mpixs_group_end_init_static(comm, ctypes.byref(h))
    return rc, h.value


def mpixs_batch_start_enqueue(batch):
    return lib().mpixs_batch_start_enqueue(batch)


def mpixs_batch_free(batch):
    h = ctypes.c_void_p(batch)
    rc = lib().mpixs_batch_free(ctypes.byref(h))
    return rc, h.value


def mpixs_send(buf, count, dt, dest, tag, comm):
    return lib().mpixs_send(ptr(buf), count, dt, dest, tag, comm)


def mpixs_recv(buf, count, dt, source, tag, comm, status=None):
    return lib().mpixs_recv(ptr(buf), count, dt, source, tag, comm, ptr(status))


def mpixs_allreduce(sendbuf, recvbuf, count, dt, op, comm):
    return lib().mpixs_allreduce(ptr(sendbuf), ptr(recvbuf), count, dt, op, comm)


def mpixs_world_get_stats(world):
    s = Stats()
    rc = lib().mpixs_world_get_stats(world, ctypes.byref(s))
    return rc, s


def mpixs_world_trace(world, max_events: int):
    """(rc, total recorded, list of TraceEvent) -- the newest max_events."""
    buf = (TraceEvent * max(1, max_events))()
    copied = ctypes.c_int64()
    total = ctypes.c_int64()
    rc = lib().mpixs_world_trace(world, buf, max_events, ctypes.byref(copied), ctypes.byref(total))
    if rc:
        return rc, 0, []
    return rc, total.value, [buf[i] for i in range(copied.value)]


def mpixs_world_reset_stats(world):
    return lib().mpixs_world_reset_stats(world)


def mpixs_error_string(rc: int) -> str:
    return lib().mpixs_error_string(rc).decode()
