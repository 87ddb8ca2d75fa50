"""ctypes binding of the native program runner (include/mpixs_driver.h) and
a small session helper that sets up a world, one HIP stream per rank and a
stream communicator per rank.

Everything here marshals arguments; all work happens in libmpixs.
"""
from __future__ import annotations

import ctypes
import os
import struct
import threading
from typing import List, Optional

import numpy as np

from . import mpixs as M

_HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER_PATH = os.path.join(_HERE, "libmpixs_driver.so")

(SEND, ISEND, RECV, IRECV, WAITALL, ALLREDUCE, MARK, GROUP_START, GROUP_END, GROUP_INIT,
 BATCH_START, BATCH_FREE, STREAM_SEND, STREAM_ISEND, STREAM_RECV, STREAM_IRECV,
 GROUP_INIT_STATIC) = range(1, 18)
BATCH_SLOTS = 8

OP_DTYPE = np.dtype([
    ("kind", "<i4"), ("comm", "<i4"), ("peer", "<i4"), ("tag", "<i4"), ("count", "<i4"),
    ("datatype", "<i4"), ("op", "<i4"), ("req", "<i4"), ("nreq", "<i4"), ("pad", "<i4"),
    ("buf", "<u8"), ("buf2", "<u8"), ("status", "<u8"),
])
assert OP_DTYPE.itemsize == 64


class DrvThread(ctypes.Structure):
    _fields_ = [("comms", ctypes.c_void_p * 16), ("ncomms", ctypes.c_int32),
                ("nmarks", ctypes.c_int32), ("hip_stream", ctypes.c_void_p),
                ("ops", ctypes.c_void_p), ("nops", ctypes.c_int64),
                ("max_reqs", ctypes.c_int32), ("nbatches", ctypes.c_int32),
                ("batches", ctypes.c_void_p)]


class DrvResult(ctypes.Structure):
    _fields_ = [("seconds", ctypes.c_double), ("first_error", ctypes.c_int32),
                ("error_thread", ctypes.c_int32), ("error_op", ctypes.c_int64),
                ("enqueue_seconds", ctypes.c_double)]


_dlib = None
_hip = None


def _hiplib():
    global _hip
    if _hip is None:
        M.lib()   # loads torch's HIP runtime first: this resolves to it
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipStreamCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        _hip.hipStreamCreateWithFlags.restype = ctypes.c_int
        _hip.hipStreamDestroy.argtypes = [ctypes.c_void_p]
        _hip.hipStreamDestroy.restype = ctypes.c_int
    return _hip


def hip_stream_create() -> int:
    """A new non-blocking HIP stream at the default priority (its own handle,
    unlike torch's pooled streams, so any number of ranks get distinct ones)."""
    s = ctypes.c_void_p()
    rc = _hiplib().hipStreamCreateWithFlags(ctypes.byref(s), 1)   # hipStreamNonBlocking
    if rc != 0:
        raise RuntimeError(f"hipStreamCreateWithFlags failed: {rc}")
    return s.value


def hip_stream_destroy(s: int) -> None:
    _hiplib().hipStreamDestroy(s)


def dlib():
    global _dlib
    if _dlib is None:
        M.lib()
        if not os.path.exists(DRIVER_PATH):
            raise RuntimeError(f"{DRIVER_PATH} is missing: run `python -m paper_2208_13707_amd.build`")
        L = ctypes.CDLL(DRIVER_PATH)
        L.mpixs_drv_run.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(DrvThread),
                                    ctypes.c_int, ctypes.POINTER(DrvResult),
                                    ctypes.POINTER(ctypes.c_double)]
        L.mpixs_drv_run.restype = ctypes.c_int
        _dlib = L
    return _dlib


def ops_array(rows) -> np.ndarray:
    """rows: list of dicts with OP_DTYPE field names (missing fields are 0)."""
    a = np.zeros(len(rows), dtype=OP_DTYPE)
    for i, r in enumerate(rows):
        for k, v in r.items():
            a[i][k] = v
    return a


def mpixs_drv_run(world, threads_ops: List[np.ndarray], comms: List[List[int]],
                  streams: List[int], mode: int = 0, nmarks: int = 0, max_reqs: int = 64,
                  batches=None):
    """batches: optional list (one per thread) of ctypes arrays of batch
    handles, kept by the caller across runs."""
    n = len(threads_ops)
    arr = (DrvThread * n)()
    keep = []
    for i in range(n):
        ops = np.ascontiguousarray(threads_ops[i], dtype=OP_DTYPE)
        keep.append(ops)
        for j, c in enumerate(comms[i]):
            arr[i].comms[j] = c
        arr[i].ncomms = len(comms[i])
        arr[i].nmarks = nmarks
        arr[i].hip_stream = streams[i]
        arr[i].ops = ops.ctypes.data
        arr[i].nops = len(ops)
        arr[i].max_reqs = max_reqs
        if batches is not None:
            arr[i].nbatches = len(batches[i])
            arr[i].batches = ctypes.addressof(batches[i])
    res = DrvResult()
    marks = np.full(max(1, n * nmarks), -1.0)
    rc = dlib().mpixs_drv_run(world, n, arr, mode, ctypes.byref(res),
                              marks.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return rc, res, marks[: n * nmarks].reshape(n, nmarks) if nmarks else None


REQ_DTYPE = np.dtype([("kind", "<i4"), ("src", "<i4"), ("dst", "<i4"), ("pad", "<i4"),
                      ("bytes", "<i8"), ("arrival_us", "<f8"), ("seed", "<u8")])
RES_DTYPE = np.dtype([("admit_us", "<f8"), ("done_us", "<f8"), ("checksum", "<u8"),
                      ("error", "<i4"), ("pad", "<i4")])


SERVE_HOST_SYNCED = 1   # MPIXS_DRV_SERVE_HOST_SYNCED
SERVE_RANK0_SUM = 2     # MPIXS_DRV_SERVE_RANK0_SUM


def mpixs_drv_serve(world, comms, streams, reqs: np.ndarray, budget_bytes: int,
                    capture=None, capture_dev: int = 0, flags: int = 0):
    """Run the serving harness; returns (rc, results array, wall seconds).
    capture: optional list of (request index, byte offset in capture_dev);
    flags: SERVE_HOST_SYNCED (host-synchronised calls instead of enqueue
    calls), SERVE_RANK0_SUM (allreduces checksummed on rank 0 only)."""
    L = dlib()
    f = L.mpixs_drv_serve
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                  ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                  ctypes.c_int64, ctypes.c_void_p, ctypes.c_int]
    f.restype = ctypes.c_int
    n = len(comms)
    ca = (ctypes.c_void_p * n)(*comms)
    sa = (ctypes.c_void_p * n)(*streams)
    reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
    res = np.zeros(max(1, len(reqs)), dtype=RES_DTYPE)
    wall = ctypes.c_double()
    cap = np.ascontiguousarray(np.array(capture or [], dtype=np.int64).reshape(-1))
    rc = f(world, n, ca, sa, reqs.ctypes.data, len(reqs), budget_bytes, res.ctypes.data,
           ctypes.byref(wall), cap.ctypes.data if cap.size else None, cap.size // 2,
           capture_dev or None, flags)
    return rc, res[: len(reqs)], wall.value


HOST_POLICIES = {"global": 0, "per_context": 1, "stream": 2}


def mpixs_drv_host_msgrate(npairs: int, policy: str, msgs_per_pair: int, window: int = 64):
    """CPU-only message-rate model (no GPU): returns (rc, msgs/s, checksum)."""
    L = dlib()
    f = L.mpixs_drv_host_msgrate
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64)]
    f.restype = ctypes.c_int
    rate = ctypes.c_double()
    ck = ctypes.c_uint64()
    rc = f(npairs, HOST_POLICIES.get(policy, -1) if isinstance(policy, str) else policy,
           msgs_per_pair, window, ctypes.byref(rate), ctypes.byref(ck))
    return rc, rate.value, ck.value


def requests_array(sched) -> np.ndarray:
    a = np.zeros(len(sched), dtype=REQ_DTYPE)
    for i, q in enumerate(sched):
        for k in ("kind", "src", "dst", "bytes", "arrival_us", "seed"):
            a[i][k] = q[k]
    return a


class Session:
    """A world of ``nranks`` ranks, each with its own torch stream, mpixs
    stream and stream communicator (created collectively from rank threads)."""

    def __init__(self, nranks: int, cfg: Optional[M.Config] = None):
        import torch
        torch.cuda.init()
        self.nranks = nranks
        self.hs = [hip_stream_create() for _ in range(nranks)]
        # persistent batch handles per rank, kept across runs
        self.batches = [(ctypes.c_void_p * BATCH_SLOTS)() for _ in range(nranks)]
        rc, self.world = M.mpixs_world_create(nranks, cfg)
        if rc:
            raise RuntimeError(f"world_create: {M.errname(rc)}")
        self.streams: List[Optional[int]] = [None] * nranks
        self.comms: List[Optional[int]] = [None] * nranks
        errs = []

        def setup(r):
            try:
                rc, wc = M.mpixs_world_comm(self.world, r)
                rc, info = M.mpixs_info_create()
                M.mpixs_info_set(info, "type", "hipStream_t")
                M.mpixs_info_set_hex(info, "value", struct.pack("<Q", self.hs[r]))
                rc, s = M.mpixs_stream_create(self.world, info)
                assert rc == 0, M.errname(rc)
                M.mpixs_info_free(info)
                self.streams[r] = s
                rc, c = M.mpixs_comm_create_with_stream(wc, s)
                assert rc == 0, M.errname(rc)
                self.comms[r] = c
            except Exception as e:  # pragma: no cover - reported below
                errs.append(repr(e))

        th = [threading.Thread(target=setup, args=(r,)) for r in range(nranks)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        if errs:
            raise RuntimeError("; ".join(errs))

    @property
    def hip_streams(self):
        return list(self.hs)

    def run(self, threads_ops, mode=0, nmarks=0, max_reqs=64):
        return mpixs_drv_run(self.world, threads_ops, [[c] for c in self.comms],
                             self.hip_streams, mode=mode, nmarks=nmarks, max_reqs=max_reqs,
                             batches=self.batches)

    def serve(self, sched, budget_bytes=8 << 30, capture=None, capture_dev=0, flags=0):
        return mpixs_drv_serve(self.world, self.comms, self.hip_streams, requests_array(sched),
                               budget_bytes, capture, capture_dev, flags)

    def stats(self):
        return M.mpixs_world_get_stats(self.world)[1]

    def stream_errors(self):
        """First asynchronous error of every rank's stream (0: none); read
        after the streams are idle."""
        out = []
        for s in self.streams:
            rc, e = M.mpixs_stream_get_error(s)
            out.append(e if rc == 0 else rc)
        return out

    def reset_stats(self):
        M.mpixs_world_reset_stats(self.world)

    def close(self):
        import torch
        torch.cuda.synchronize()
        for r in range(self.nranks):
            for h in self.batches[r]:
                if h:
                    M.mpixs_batch_free(h)
            M.mpixs_comm_free(self.comms[r])
            M.mpixs_stream_free(self.streams[r])
        M.mpixs_world_free(self.world)
        for s in self.hs:
            hip_stream_destroy(s)


class NTo1Session:
    """Two ranks for an N-to-1 pattern (§3.5): rank 0 has ``nsend`` threads,
    each with its own stream; rank 1 has one polling thread with one stream.
    Communicators: ``mux`` (one multiplex communicator over all of them, per
    rank) and, for comparison, ``pair[i]`` (one stream communicator joining
    sender stream i and the polling stream)."""

    def __init__(self, nsend: int, cfg: Optional[M.Config] = None):
        import torch
        torch.cuda.init()
        self.nsend = nsend
        self.hs0 = [hip_stream_create() for _ in range(nsend)]
        self.hs1 = hip_stream_create()
        rc, self.world = M.mpixs_world_create(2, cfg)
        if rc:
            raise RuntimeError(f"world_create: {M.errname(rc)}")
        self.s0, self.s1 = [], None
        self.mux = [None, None]
        self.pair = [[None, None] for _ in range(nsend)]
        errs = []

        def mk(h):
            rc, info = M.mpixs_info_create()
            M.mpixs_info_set(info, "type", "hipStream_t")
            M.mpixs_info_set_hex(info, "value", struct.pack("<Q", h))
            rc, s = M.mpixs_stream_create(self.world, info)
            assert rc == 0, M.errname(rc)
            M.mpixs_info_free(info)
            return s

        def setup(r):
            try:
                rc, wc = M.mpixs_world_comm(self.world, r)
                if r == 0:
                    self.s0 = [mk(h) for h in self.hs0]
                    mine = self.s0
                else:
                    self.s1 = mk(self.hs1)
                    mine = [self.s1]
                rc, c = M.mpixs_comm_create_multiplex(wc, mine)
                assert rc == 0, M.errname(rc)
                self.mux[r] = c
                for i in range(nsend):
                    rc, c = M.mpixs_comm_create_with_stream(wc, self.s0[i] if r == 0 else self.s1)
                    assert rc == 0, M.errname(rc)
                    self.pair[i][r] = c
            except Exception as e:  # pragma: no cover - reported below
                errs.append(repr(e))

        th = [threading.Thread(target=setup, args=(r,)) for r in range(2)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        if errs:
            raise RuntimeError("; ".join(errs))

    def run(self, sender_ops, receiver_ops, mode=0, max_reqs=64):
        """sender_ops[i]: thread i of rank 0 (communicators [mux, pair[i]]);
        receiver_ops: the polling thread (communicators [mux, pair[0..n-1]])."""
        comms = [[self.mux[0], self.pair[i][0]] for i in range(self.nsend)]
        comms.append([self.mux[1]] + [self.pair[i][1] for i in range(self.nsend)])
        return mpixs_drv_run(self.world, list(sender_ops) + [receiver_ops], comms,
                             list(self.hs0) + [self.hs1], mode=mode, max_reqs=max_reqs)

    def stream_errors(self):
        """First asynchronous error of every stream (0: none)."""
        out = []
        for s in list(self.s0) + [self.s1]:
            rc, e = M.mpixs_stream_get_error(s)
            out.append(e if rc == 0 else rc)
        return out

    def close(self):
        import torch
        torch.cuda.synchronize()
        for r in range(2):
            M.mpixs_comm_free(self.mux[r])
            for i in range(self.nsend):
                M.mpixs_comm_free(self.pair[i][r])
        for s in self.s0 + [self.s1]:
            M.mpixs_stream_free(s)
        M.mpixs_world_free(self.world)
        for h in self.hs0 + [self.hs1]:
            hip_stream_destroy(h)
