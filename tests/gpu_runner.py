"""Run a workloads.Program on the GPU through the libmpixs Python binding.

One Python thread per (rank, thread) issues that thread's operations through
the C ABI (ctypes releases the GIL around every call); user kernels of the
program are plain torch operations on the rank's stream.  Buffers and
statuses live in device memory.  Returns the same fields as the oracle's
simulator so the two can be compared byte for byte.
"""
from __future__ import annotations

import struct
import sys
import threading
import traceback
from dataclasses import dataclass
from typing import Dict, List, Optional, Tuple

import numpy as np

from workloads.program import (
    IN_PLACE, Allreduce, GroupEnd, GroupInit, GroupStart, Program, Recv, Send, Start, User, Wait,
)


@dataclass
class GpuResult:
    buffers: List[Dict[str, np.ndarray]]
    statuses: List[Dict[str, Tuple[int, int, str, int]]]
    sync_errors: List[List[Tuple[int, int, str]]]
    stream_errors: List[List[str]]
    stats: object
    status_index: object = None      # per rank: status name -> sender's stream index


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


class _Types:
    """Constructor trees -> committed libmpixs datatypes (cached)."""

    def __init__(self, M):
        self.M = M
        self.cache = {}
        self.lock = threading.Lock()

    def _build(self, tree):
        M = self.M
        if isinstance(tree, str):
            return M.BASIC.get(tree, 0)
        kind = tree[0]
        if kind == "contiguous":
            rc, t = M.mpixs_type_contiguous(tree[1], self._build(tree[2]))
        elif kind == "vector":
            rc, t = M.mpixs_type_vector(tree[1], tree[2], tree[3], self._build(tree[4]))
        elif kind == "indexed":
            rc, t = M.mpixs_type_indexed(list(tree[1]), list(tree[2]), self._build(tree[3]))
        else:
            return 0
        return t if rc == 0 else 0

    def get(self, tree):
        key = repr(tree)
        with self.lock:
            if key not in self.cache:
                t = self._build(tree)
                if t and not isinstance(tree, str):
                    rc, t2 = self.M.mpixs_type_commit(t)
                    t = t2 if rc == 0 else 0
                self.cache[key] = t
            return self.cache[key]


def _status_layout(p: Program):
    """Per rank: name -> slot index; Wait ops with statuses get contiguous blocks."""
    layout, wait_block = [], []
    for r in range(p.nranks):
        names: Dict[str, int] = {}
        blocks: Dict[Tuple[int, int], int] = {}
        n = 0
        for t, lst in enumerate(p.ops[r]):
            for i, o in enumerate(lst):
                if isinstance(o, Recv) and o.status is not None:
                    names[o.status] = n
                    n += 1
                elif isinstance(o, Wait) and any(s is not None for s in o.statuses):
                    blocks[(t, i)] = n
                    for j, s in enumerate(o.statuses):
                        if s is not None:
                            names[s] = n + j
                    n += len(o.statuses)
        layout.append((names, n))
        wait_block.append(blocks)
    return layout, wait_block


def run_program(p: Program, cfg=None, host_synced: bool = False, timeout_s: float = 120.0,
                stats: bool = False) -> GpuResult:
    import torch
    from paper_2208_13707_amd import mpixs as M

    dev = torch.device("cuda:0")
    N = p.nranks
    dbufs = [{k: torch.from_numpy(v.copy()).to(dev) for k, v in b.items()} for b in p.buffers]
    layout, wait_block = _status_layout(p)
    dstat = [torch.full((max(1, n) * M.STATUS_BYTES,), 0xEE, dtype=torch.uint8, device=dev)
             for _, n in layout]
    from paper_2208_13707_amd import driver as D
    hip_streams = [[D.hip_stream_create() for _ in range(p.streams_per_rank)] for _ in range(N)]
    tstreams = [[torch.cuda.ExternalStream(h, device=dev) for h in row] for row in hip_streams]
    torch.cuda.synchronize()

    if p.matching == "queue":
        # ordered-queue matching (wildcards allowed)
        base = cfg
        cfg = M.Config()
        if base is not None:
            for name, _ in M.Config._fields_:
                setattr(cfg, name, getattr(base, name))
        cfg.matching = 1
    rc, world = M.mpixs_world_create(N, cfg)
    assert rc == 0, M.errname(rc)
    types = _Types(M)
    mstreams: List[List[Optional[int]]] = [[None] * p.streams_per_rank for _ in range(N)]
    comms: List[List[Optional[int]]] = [[None] * p.ncomms for _ in range(N)]
    failures: List[str] = []

    def setup(r):
        try:
            rc, wc = M.mpixs_world_comm(world, r)
            assert rc == 0
            for s in range(p.streams_per_rank):
                rc, info = M.mpixs_info_create()
                assert rc == 0
                M.mpixs_info_set(info, "type", "hipStream_t")
                M.mpixs_info_set_hex(info, "value",
                                     struct.pack("<Q", tstreams[r][s].cuda_stream))
                rc, h = M.mpixs_stream_create(world, info)
                assert rc == 0, M.errname(rc)
                M.mpixs_info_free(info)
                mstreams[r][s] = h
            for c in range(p.ncomms):
                st = p.comm_streams[c][r]
                if isinstance(st, list):
                    rc, h = M.mpixs_comm_create_multiplex(wc, [mstreams[r][s] for s in st])
                else:
                    rc, h = M.mpixs_comm_create_with_stream(
                        wc, mstreams[r][st] if st is not None else None)
                assert rc == 0, M.errname(rc)
                comms[r][c] = h
        except Exception:
            failures.append(f"setup rank {r}:\n{traceback.format_exc()}")

    th = [threading.Thread(target=setup, args=(r,)) for r in range(N)]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout_s)
    if failures:
        raise RuntimeError("\n".join(failures))

    sync_errors: List[List[Tuple[int, int, str]]] = [[] for _ in range(N)]
    requests: List[Dict[str, int]] = [dict() for _ in range(N)]
    batches: List[Dict[str, Optional[int]]] = [dict() for _ in range(N)]
    err_lock = threading.Lock()

    def comm_of(r, c):
        if 0 <= c < p.ncomms:
            return comms[r][c]
        return None

    def bufptr(r, name, off):
        return dbufs[r][name].data_ptr() + off

    def status_ptr(r, name):
        if name is None:
            return None
        return dstat[r].data_ptr() + layout[r][0][name] * M.STATUS_BYTES

    def user(r, o: User):
        fn = o.fn
        with torch.cuda.stream(tstreams[r][o.stream]):
            if fn[0] == "add_const_i32":
                _, b, off, n, c = fn
                x = dbufs[r][b][off: off + 4 * n].view(torch.int32)
                x.add_(c)
            elif fn[0] == "saxpy_f32":
                _, xb, xoff, yb, yoff, n, a = fn
                x = dbufs[r][xb][xoff: xoff + 4 * n].view(torch.float32)
                y = dbufs[r][yb][yoff: yoff + 4 * n].view(torch.float32)
                ax = x * a                       # rounded product
                y.add_(ax)                       # rounded sum
            elif fn[0] == "add_rows_f32":
                _, db, doff, sb, soff, rows, re, lo, hi = fn
                d = dbufs[r][db][doff: doff + 4 * rows * re].view(torch.float32).view(rows, re)
                s = dbufs[r][sb][soff: soff + 4 * rows * re].view(torch.float32).view(rows, re)
                d[:, lo:hi] += s[:, lo:hi]
            else:
                raise ValueError(fn)

    def record(r, t, i, rc):
        if rc != 0:
            with err_lock:
                sync_errors[r].append((t, i, M.errname(rc)))

    def worker(r, t):
        try:
            for i, o in enumerate(p.ops[r][t]):
                if isinstance(o, (Send, Recv)) and (o.src_idx is not None or o.dst_idx is not None):
                    # index-addressed call of a multiplex communicator
                    dt = types.get(o.dtype)
                    c = comm_of(r, o.comm)
                    si = o.src_idx if o.src_idx is not None else -99
                    di = o.dst_idx if o.dst_idx is not None else -99
                    if isinstance(o, Send) and o.req is None:
                        rc = M.mpixs_stream_send_enqueue(bufptr(r, o.buf, o.off), o.count, dt,
                                                         o.dest, o.tag, c, si, di)
                    elif isinstance(o, Send):
                        rc, h = M.mpixs_stream_isend_enqueue(bufptr(r, o.buf, o.off), o.count, dt,
                                                             o.dest, o.tag, c, si, di)
                        if rc == 0:
                            requests[r][o.req] = h
                    elif o.req is None:
                        rc = M.mpixs_stream_recv_enqueue(bufptr(r, o.buf, o.off), o.count, dt,
                                                         o.source, o.tag, c, si, di,
                                                         status_ptr(r, o.status))
                    else:
                        rc, h = M.mpixs_stream_irecv_enqueue(bufptr(r, o.buf, o.off), o.count, dt,
                                                             o.source, o.tag, c, si, di)
                        if rc == 0:
                            requests[r][o.req] = h
                    record(r, t, i, rc)
                elif isinstance(o, Send):
                    dt = types.get(o.dtype)
                    c = comm_of(r, o.comm)
                    if host_synced:
                        rc = M.mpixs_send(bufptr(r, o.buf, o.off), o.count, dt, o.dest, o.tag, c)
                    elif o.req is None:
                        rc = M.mpixs_send_enqueue(bufptr(r, o.buf, o.off), o.count, dt, o.dest,
                                                  o.tag, c)
                    else:
                        rc, h = M.mpixs_isend_enqueue(bufptr(r, o.buf, o.off), o.count, dt, o.dest,
                                                      o.tag, c)
                        if rc == 0:
                            requests[r][o.req] = h
                    record(r, t, i, rc)
                elif isinstance(o, Recv):
                    dt = types.get(o.dtype)
                    c = comm_of(r, o.comm)
                    if host_synced:
                        rc = M.mpixs_recv(bufptr(r, o.buf, o.off), o.count, dt, o.source, o.tag, c,
                                          status_ptr(r, o.status))
                    elif o.req is None:
                        rc = M.mpixs_recv_enqueue(bufptr(r, o.buf, o.off), o.count, dt, o.source,
                                                  o.tag, c, status_ptr(r, o.status))
                    else:
                        rc, h = M.mpixs_irecv_enqueue(bufptr(r, o.buf, o.off), o.count, dt,
                                                      o.source, o.tag, c)
                        if rc == 0:
                            requests[r][o.req] = h
                    record(r, t, i, rc)
                elif isinstance(o, Wait):
                    hs = [requests[r].get(n, 0) for n in o.reqs]
                    if host_synced:
                        continue
                    blk = wait_block[r].get((t, i))
                    sp = None if blk is None else dstat[r].data_ptr() + blk * M.STATUS_BYTES
                    if len(hs) == 1:
                        rc, _ = M.mpixs_wait_enqueue(hs[0] or None, sp)
                    else:
                        rc, _ = M.mpixs_waitall_enqueue(hs, sp)
                    if rc == 0:
                        for n in o.reqs:
                            requests[r].pop(n, None)
                    record(r, t, i, rc)
                elif isinstance(o, Allreduce):
                    dt = M.BASIC.get(o.dtype, 99)
                    if o.dtype in ("uint8", "int8"):
                        dt = M.BASIC[o.dtype]
                    op = M.OPS.get(o.op, 99)
                    sb = M.IN_PLACE if o.sendbuf == IN_PLACE else bufptr(r, o.sendbuf, o.soff)
                    c = comm_of(r, o.comm)
                    fn = M.mpixs_allreduce if host_synced else M.mpixs_allreduce_enqueue
                    rc = fn(sb, bufptr(r, o.recvbuf, o.roff), o.count, dt, op, c)
                    record(r, t, i, rc)
                elif isinstance(o, User):
                    user(r, o)
                elif isinstance(o, GroupStart):
                    record(r, t, i, M.mpixs_group_start(comm_of(r, o.comm)))
                elif isinstance(o, GroupEnd):
                    record(r, t, i, M.mpixs_group_end(comm_of(r, o.comm)))
                elif isinstance(o, GroupInit):
                    rc, h = M.mpixs_group_end_init(comm_of(r, o.comm))
                    batches[r][o.batch] = h
                    record(r, t, i, rc)
                elif isinstance(o, Start):
                    record(r, t, i, M.mpixs_batch_start_enqueue(batches[r].get(o.batch)))
                else:
                    raise ValueError(o)
        except Exception:
            failures.append(f"rank {r} thread {t}:\n{traceback.format_exc()}")

    th = [threading.Thread(target=worker, args=(r, t), daemon=True)
          for r in range(N) for t in range(len(p.ops[r]))]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout_s)
    hung = [x for x in th if x.is_alive()]
    if hung:
        M.mpixs_world_abort(world)
        for x in hung:
            x.join(30)
        failures.append(f"{len(hung)} threads did not finish within {timeout_s}s (world aborted)")
    rc = M.mpixs_world_wait(world, int(timeout_s * 1000))
    if rc != 0:
        M.mpixs_world_abort(world)
        M.mpixs_world_wait(world, 60000)
        failures.append(f"streams did not drain: {M.errname(rc)}")
    # the rank streams alone: results are read on torch's stream afterwards,
    # which the stream contract allows without a device-wide synchronisation
    for row in tstreams:
        for ts in row:
            ts.synchronize()
    if failures:
        raise RuntimeError("\n".join(failures))

    out_bufs = [{k: v.cpu().numpy().copy() for k, v in b.items()} for b in dbufs]
    statuses, status_index = [], []
    for r in range(N):
        raw = dstat[r].cpu().numpy().tobytes()
        d, di = {}, {}
        for name, idx in layout[r][0].items():
            src, tag, err, sidx, cnt = struct.unpack_from("<iiiiq", raw, idx * M.STATUS_BYTES)
            d[name] = (src, tag, M.errname(err), cnt)
            di[name] = sidx
        statuses.append(d)
        status_index.append(di)
    stream_errors = []
    for r in range(N):
        errs = []
        for s in range(p.streams_per_rank):
            rc, e = M.mpixs_stream_get_error(mstreams[r][s])
            errs.append(M.errname(e))
        stream_errors.append(errs)
    st = None
    if stats:
        _, st = M.mpixs_world_get_stats(world)
    for r in range(N):
        for h in batches[r].values():
            if h:
                assert M.mpixs_batch_free(h)[0] == 0
        for c in range(p.ncomms):
            assert M.mpixs_comm_free(comms[r][c]) == 0
        for s in range(p.streams_per_rank):
            rc = M.mpixs_stream_free(mstreams[r][s])
            assert rc == 0, M.errname(rc)
    assert M.mpixs_world_free(world) == 0
    for row in hip_streams:
        for h in row:
            D.hip_stream_destroy(h)
    return GpuResult(out_bufs, statuses, [sorted(e) for e in sync_errors], stream_errors, st,
                     status_index)


def compare(p: Program, gpu: GpuResult, ref, check_statuses: bool = True) -> List[str]:
    """Differences between a GPU result and the oracle's (empty when equal)."""
    diffs = []
    for r in range(p.nranks):
        for k, v in ref.buffers[r].items():
            g = gpu.buffers[r][k]
            if not np.array_equal(g, v):
                bad = np.nonzero(g != v)[0]
                diffs.append(f"rank {r} buffer {k}: {bad.size} bytes differ, first at {bad[:5]}")
        if check_statuses:
            for name, val in ref.statuses[r].items():
                if gpu.statuses[r].get(name) != val:
                    diffs.append(f"rank {r} status {name}: gpu {gpu.statuses[r].get(name)} "
                                 f"oracle {val}")
        if sorted(ref.sync_errors[r]) != gpu.sync_errors[r]:
            diffs.append(f"rank {r} sync errors: gpu {gpu.sync_errors[r]} oracle "
                         f"{sorted(ref.sync_errors[r])}")
    return diffs

