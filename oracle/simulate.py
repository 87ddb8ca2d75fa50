"""Deterministic simulator of enqueue programs (oracle; test infrastructure only).

What it states, and where the paper fixes it:

* Each stream is a strictly serial local context (§3.1), driven by one host
  thread: the operations a thread issues take effect in its program order.
  Threads of different ranks, and different threads of one rank, progress
  independently.
* Matching order is an MPI outcome, delivery order is not (§2.1): with no
  wildcards, the k-th send that rank s issues on channel (comm, s, d, tag)
  matches the k-th receive that rank d issues on the same channel.
  Communicators are matched independently, and so are tags (§2.1).
* Enqueue semantics (§3.4): a send or isend reads its buffer only after the
  earlier operations of its stream are done; a blocking send completes when
  its buffer may be reused, an isend lets later operations proceed until the
  matching wait; a receive's data is in place when the receive (or its wait)
  completes.  Waitall takes requests of one stream only (§3.4).
* Collectives extend the enqueue interface (§3.4): the k-th allreduce that
  each rank issues on a communicator forms one instance, complete once all
  ranks reached it; its result is the canonical-order fold (see reduce.py).
* Enqueue calls on a communicator without a local GPU stream are an error
  (§3.4).
* Matching with wildcards (programs with matching = "queue"): MPI's rule
  with posted and unexpected queues per destination -- a send meets the
  earliest posted receive that accepts its (source, tag), a receive (source
  may be ANY_SOURCE, tag ANY_TAG) meets the earliest unmatched send to it
  that it accepts, else the operation waits in its queue.  "Earliest" is the
  order in which the operations are issued; messages of one sender keep
  their order.  When several senders compete for a wildcard receive the
  result depends on that order (in MPI and on the GPU alike), so such
  programs are compared by invariants, not byte for byte.  Wildcards are not
  allowed inside groups.
* Multiplex stream communicators (§3.5): every rank attaches several
  streams, addressed by index; a send names its own index and the
  receiver's, a receive its own index and the sender's (or ANY_INDEX).
  Matching is the queue matching above, per destination (rank, index).
  Ordinary calls, allreduce and groups on such a communicator are ERR_COMM
  (it has no single stream), and index calls on other communicators too.
* Groups (a batching extension): between GroupStart and GroupEnd on a
  communicator a rank's sends and receives on it are posted but do not
  block and do not move data; GroupEnd is collective (instance k = the k-th
  GroupEnd of each rank on the communicator) and, once every rank reached
  it, moves all of the instance's messages.  A grouped message whose peer
  operation is not grouped in the same instance makes the whole instance
  fail: no message of it moves and every rank's GroupEnd reports ERR_ARG.
  A wait on a grouped request inside its group delivers the status at the
  group's end.  Allreduces inside a group are recorded too: the i-th grouped
  allreduce of every rank forms the instance's i-th reduction, run at the
  group's end after its messages have moved, in order; ranks that grouped
  different numbers of allreduces, or i-th calls that differ in count, type
  or operation, fail the instance like an unmatched message.
* Persistent groups (the same extension, with MPI's persistent-request
  model of init once, start many times): a group closed by GroupInit is
  recorded, not run.  GroupInit is collective; it fails with ERR_ARG on
  every rank when a recorded send or receive has no partner among all ranks'
  recorded operations of that group or a request created in it is not
  waited for inside it, and a Start of a failed (or unknown) batch is
  ERR_REQUEST.  The j-th Start of every rank forms run j, which behaves
  exactly as if each rank had issued GroupStart, its recorded operations and
  GroupEnd at that point: payloads are the send buffers' contents when the
  run happens.

Readings where the paper is silent (each is listed in the design notes):

* Blocking sends have synchronous-send semantics here (complete only when
  matched and transferred), the strictest legal reading.  A program that
  completes under it is "safe"; one that cannot is reported as a deadlock.
* An isend's data is taken at the moment it is posted; changing the buffer
  before the wait is erroneous, so any later moment gives the same bytes.
* Receive checks, in this order: when both the message and the receive
  buffer hold data and their basic types differ, the error is ERR_TYPE and
  nothing is written (count 0); when the message holds more bytes than the
  receive buffer, the leading bytes that fit are written, the error is
  ERR_TRUNCATE and the count is the receive capacity; else the count is the
  message size in bytes.
* Invalid arguments are reported when the op is issued and the op then has
  no effect at all.  Checks run in this order: communicator (ERR_COMM),
  count (ERR_COUNT), datatype (ERR_TYPE), peer rank (ERR_RANK, also for the
  any-source wildcard where wildcards are not allowed), tag (ERR_TAG,
  likewise), stream indices of a multiplex communicator (ERR_RANK),
  overlapping receive typemap (ERR_TYPE); for allreduce: communicator, count,
  datatype (basic types only), operation (ERR_OP); for wait / waitall:
  unknown request (ERR_REQUEST), requests of different streams (ERR_STREAM).
  The paper prints no example of these codes, so the order is this
  simulator's reading; the tests pin that the simulator follows it, with
  expected codes written out by hand for fixed programs of erroneous calls
  (and that such calls move nothing).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import reduce as red
from . import typemap as tm
from workloads.program import (
    ANY_INDEX, ANY_SOURCE, ANY_TAG, IN_PLACE, Allreduce, GroupEnd, GroupInit, GroupStart, Program,
    Recv, Send,
    Start, User, Wait,
)

SUCCESS = "SUCCESS"


@dataclass
class _SendRec:
    rank: int
    tag: int
    basic: str
    payload: Optional[np.ndarray]
    done: bool = False
    group: Optional[Tuple[int, int]] = None     # (comm, instance) when grouped
    src: Optional[Tuple[str, int, int, object]] = None   # (buf, off, count, typemap)
    idx: int = 0                                # sender's stream index (multiplex)


@dataclass
class _RecvRec:
    rank: int
    buf: str
    off: int
    count: int
    t: tm.Typemap
    done: bool = False
    status: Optional[Tuple[int, int, str, int]] = None
    group: Optional[Tuple[int, int]] = None
    want: Tuple[int, int, int] = (0, 0, 0)       # queue matching: (source, index, tag) accepted


@dataclass
class _Chan:
    sends: Dict[int, _SendRec] = field(default_factory=dict)
    recvs: Dict[int, _RecvRec] = field(default_factory=dict)
    nsend: int = 0
    nrecv: int = 0


@dataclass
class Result:
    buffers: List[Dict[str, np.ndarray]]
    statuses: List[Dict[str, Tuple[int, int, str, int]]]
    sync_errors: List[List[Tuple[int, int, str]]]     # per rank: (thread, op index, error)
    match_log: List[Tuple[int, int, int, int, int]]   # (comm, src, dst, tag, k)
    deadlock: bool
    blocked: List[Tuple[int, int, int]]               # (rank, thread, op index) left blocked


class _Context:
    def __init__(self, rank: int, thread: int, ops):
        self.rank = rank
        self.thread = thread
        self.ops = ops
        self.pc = 0
        self.pending = None          # record the current blocking op waits on


def _check_p2p(p: Program, rank: int, op) -> Optional[str]:
    if not (0 <= op.comm < p.ncomms):
        return "ERR_COMM"
    mp = p.multiplex(op.comm)
    if mp != (op.src_idx is not None or op.dst_idx is not None):
        return "ERR_COMM"        # an ordinary call on a multiplex communicator, or vice versa
    if not mp and p.stream_of(rank, op.comm) is None:
        return "ERR_COMM"
    if op.count < 0:
        return "ERR_COUNT"
    try:
        t = tm.build(op.dtype)
    except tm.TypeError_:
        return "ERR_TYPE"
    recv = isinstance(op, Recv)
    peer = op.dest if isinstance(op, Send) else op.source
    wild = recv and (p.matching == "queue" or mp)
    if not (0 <= peer < p.nranks) and not (wild and peer == ANY_SOURCE):
        return "ERR_RANK"
    if op.tag < 0 and not (wild and op.tag == ANY_TAG):
        return "ERR_TAG"
    if mp:
        streams = p.comm_streams[op.comm]
        local = op.dst_idx if recv else op.src_idx
        remote = op.src_idx if recv else op.dst_idx
        if local is None or not (0 <= local < len(streams[rank])):
            return "ERR_RANK"
        if recv and remote == ANY_INDEX:
            pass
        elif recv and peer == ANY_SOURCE:
            if remote is None or remote < 0:
                return "ERR_RANK"
        elif remote is None or not (0 <= remote < len(streams[peer])):
            return "ERR_RANK"
    if isinstance(op, Recv) and tm.overlaps(t, op.count):
        return "ERR_TYPE"
    return None


def _colls_agree(colls, nranks) -> bool:
    """The grouped allreduces of an instance form collectives: every rank made
    as many, and the i-th of each rank agree in count, type and operation."""
    lists = [colls.get(q, []) for q in range(nranks)]
    if len({len(x) for x in lists}) > 1:
        return False
    for i in range(len(lists[0])):
        if len({(x[i].count, x[i].dtype, x[i].op) for x in lists}) > 1:
            return False
    return True


def _check_allreduce(p: Program, rank: int, op: Allreduce) -> Optional[str]:
    if not (0 <= op.comm < p.ncomms) or p.stream_of(rank, op.comm) is None:
        return "ERR_COMM"
    if op.count < 0:
        return "ERR_COUNT"
    if op.dtype not in red.NP_DTYPE or op.dtype in ("uint8", "int8"):
        return "ERR_TYPE"
    if op.op not in red.OPS:
        return "ERR_OP"
    return None


def _apply_user(bufs: Dict[str, np.ndarray], fn: tuple) -> None:
    """Deterministic user kernels (the application's own work on its stream)."""
    name = fn[0]
    if name == "add_const_i32":
        _, b, off, n, c = fn
        x = bufs[b][off: off + 4 * n].view(np.int32)
        x += np.int32(c)
    elif name == "saxpy_f32":
        _, xb, xoff, yb, yoff, n, a = fn
        x = bufs[xb][xoff: xoff + 4 * n].view(np.float32)
        y = bufs[yb][yoff: yoff + 4 * n].view(np.float32)
        y[:] = (np.float32(a) * x) + y      # two roundings, as the GPU kernel
    elif name == "add_rows_f32":
        _, db, doff, sb, soff, rows, row_elems, lo, hi = fn
        d = bufs[db][doff: doff + 4 * rows * row_elems].view(np.float32).reshape(rows, row_elems)
        s = bufs[sb][soff: soff + 4 * rows * row_elems].view(np.float32).reshape(rows, row_elems)
        d[:, lo:hi] += s[:, lo:hi]
    else:
        raise ValueError(f"unknown user kernel {name!r}")


def run(p: Program, max_rounds: int = 10_000_000) -> Result:
    bufs = p.copy_buffers()
    statuses: List[Dict[str, Tuple[int, int, str, int]]] = [dict() for _ in range(p.nranks)]
    sync_errors: List[List[Tuple[int, int, str]]] = [[] for _ in range(p.nranks)]
    match_log: List[Tuple[int, int, int, int, int]] = []
    chans: Dict[Tuple[int, int, int, int], _Chan] = {}
    requests: List[Dict[str, Tuple[object, int]]] = [dict() for _ in range(p.nranks)]
    coll_next: Dict[Tuple[int, int], int] = {}          # (comm, rank) -> next instance
    coll: Dict[Tuple[int, int], Dict[int, Allreduce]] = {}
    coll_done: Dict[Tuple[int, int], bool] = {}
    group_open: Dict[Tuple[int, int], Tuple[int, int]] = {}    # (rank, comm) -> (comm, inst)
    group_next: Dict[Tuple[int, int], int] = {}                # (rank, comm) -> next instance
    group_arrived: Dict[Tuple[int, int], set] = {}
    group_msgs: Dict[Tuple[int, int], list] = {}
    group_ok: Dict[Tuple[int, int], bool] = {}
    group_after: Dict[Tuple[int, int], list] = {}
    group_colls: Dict[tuple, Dict[int, list]] = {}             # grp -> rank -> allreduces
    # persistent groups
    persist_open: Dict[Tuple[int, int], str] = {}              # (rank, comm) -> batch name
    batch_ops: Dict[Tuple[int, str], list] = {}                # (rank, batch) -> recorded ops
    batch_arrived: Dict[str, set] = {}
    batch_bad: Dict[str, bool] = {}
    batch_ok: Dict[str, bool] = {}
    batch_runs: Dict[Tuple[int, str], int] = {}

    def terminators(ops):
        """GroupStart index -> the op that closes that group (GroupEnd or
        GroupInit on the same communicator), found by scanning ahead."""
        out, open_ = {}, {}
        for i, o in enumerate(ops):
            if isinstance(o, GroupStart) and o.comm not in open_:
                open_[o.comm] = i
            elif isinstance(o, (GroupEnd, GroupInit)) and o.comm in open_:
                out[open_.pop(o.comm)] = o
        return out

    def record_grouped(rank, op, grp):
        """Post a send / receive / wait / allreduce inside group ``grp`` (a
        one-shot group instance, or a run of a persistent batch)."""
        if isinstance(op, Allreduce):
            group_colls.setdefault(grp, {}).setdefault(rank, []).append(op)
            return
        if isinstance(op, Wait):
            # each request's status arrives at the end of its own group
            for n, st_name in zip(op.reqs, op.statuses):
                r = requests[rank].pop(n)[0]
                if not isinstance(r, _RecvRec) or st_name is None:
                    continue
                if r.group in group_ok:
                    if group_ok[r.group]:
                        statuses[rank][st_name] = r.status
                else:
                    group_after.setdefault(r.group, []).append(
                        lambda ok, r=r, st_name=st_name, rank=rank:
                        statuses[rank].__setitem__(st_name, r.status) if ok else None)
            return
        rec = post_send(rank, op, grp) if isinstance(op, Send) else post_recv(rank, op, grp)
        if op.req is not None:
            requests[rank][op.req] = (rec, p.stream_of(rank, op.comm))
        elif isinstance(op, Recv) and op.status is not None:
            name = op.status
            group_after.setdefault(grp, []).append(
                lambda ok, rec=rec, name=name, rank=rank:
                statuses[rank].__setitem__(name, rec.status) if ok else None)

    def init_batch(name):
        """Every rank reached GroupInit of ``name``: accept it if each
        recorded send has a recorded partner (per channel, equal counts)."""
        count: Dict[tuple, int] = {}
        for (rank, b), ops in batch_ops.items():
            if b != name:
                continue
            for o in ops:
                if isinstance(o, Send):
                    key = (o.comm, rank, o.dest, o.tag)
                    count[key] = count.get(key, 0) + 1
                elif isinstance(o, Recv):
                    key = (o.comm, o.source, rank, o.tag)
                    count[key] = count.get(key, 0) - 1
        colls = {rank: [o for o in ops if isinstance(o, Allreduce)]
                 for (rank, b), ops in batch_ops.items() if b == name}
        batch_ok[name] = (not batch_bad.get(name, False) and all(v == 0 for v in count.values())
                          and _colls_agree(colls, p.nranks))

    def chan(key):
        if key not in chans:
            chans[key] = _Chan()
        return chans[key]

    def transfer(key, k):
        move(chans[key].sends[k], chans[key].recvs[k], key, k)

    def move(s, r, key, k):
        """Unpack send s into receive r (the receive checks of the module
        docstring) and log the match."""
        if s.payload is None:
            buf, off, count, t = s.src
            s.payload = tm.pack(bufs[s.rank][buf], off, count, t)
        cap = r.count * r.t.size
        nbytes = int(s.payload.size)
        if nbytes > 0 and cap > 0 and s.basic != r.t.basic:
            err, written = "ERR_TYPE", 0
        elif nbytes > cap:
            err, written = "ERR_TRUNCATE", cap
        else:
            err, written = SUCCESS, nbytes
        if written:
            tm.unpack(bufs[r.rank][r.buf], r.off, r.count, r.t, s.payload[:written])
        r.status = (s.rank, s.tag, err, written)
        s.done = r.done = True
        match_log.append((key[0], key[1], key[2], key[3], k))

    # (comm, dst, dst stream index) -> (unexpected, posted)
    queues: Dict[Tuple[int, int, int], Tuple[list, list]] = {}
    qcount: Dict[Tuple[int, int, int, int], int] = {}

    def queue_match(s, r, comm):
        key = (comm, s.rank, r.rank, s.tag)
        k = qcount.get(key, 0)
        qcount[key] = k + 1
        move(s, r, key, k)

    def accepts(r, s):
        src, idx, tag = r.want
        return src in (ANY_SOURCE, s.rank) and idx in (ANY_INDEX, s.idx) and tag in (ANY_TAG, s.tag)

    def post_send_q(rank, op: Send) -> _SendRec:
        t = tm.build(op.dtype)
        rec = _SendRec(rank, op.tag, t.basic, tm.pack(bufs[rank][op.buf], op.off, op.count, t),
                       idx=op.src_idx or 0)
        unexpected, posted = queues.setdefault((op.comm, op.dest, op.dst_idx or 0), ([], []))
        for i, r in enumerate(posted):
            if accepts(r, rec):
                del posted[i]
                queue_match(rec, r, op.comm)
                return rec
        unexpected.append(rec)
        return rec

    def post_recv_q(rank, op: Recv) -> _RecvRec:
        t = tm.build(op.dtype)
        rec = _RecvRec(rank, op.buf, op.off, op.count, t,
                       want=(op.source, op.src_idx if op.src_idx is not None else 0, op.tag))
        unexpected, posted = queues.setdefault((op.comm, rank, op.dst_idx or 0), ([], []))
        for i, s in enumerate(unexpected):
            if accepts(rec, s):
                del unexpected[i]
                queue_match(s, rec, op.comm)
                return rec
        posted.append(rec)
        return rec

    def post_send(rank, op: Send, group=None) -> _SendRec:
        t = tm.build(op.dtype)
        key = (op.comm, rank, op.dest, op.tag)
        c = chan(key)
        if group is None:
            rec = _SendRec(rank, op.tag, t.basic, tm.pack(bufs[rank][op.buf], op.off, op.count, t))
        else:
            rec = _SendRec(rank, op.tag, t.basic, None, group=group,
                           src=(op.buf, op.off, op.count, t))
        k = c.nsend
        c.nsend += 1
        c.sends[k] = rec
        if group is None and k in c.recvs and c.recvs[k].group is None:
            transfer(key, k)
        elif group is not None:
            group_msgs.setdefault(group, []).append((key, k))
        return rec

    def post_recv(rank, op: Recv, group=None) -> _RecvRec:
        t = tm.build(op.dtype)
        key = (op.comm, op.source, rank, op.tag)
        c = chan(key)
        rec = _RecvRec(rank, op.buf, op.off, op.count, t, group=group)
        k = c.nrecv
        c.nrecv += 1
        c.recvs[k] = rec
        if group is None and k in c.sends and c.sends[k].group is None:
            transfer(key, k)
        elif group is not None:
            group_msgs.setdefault(group, []).append((key, k))
        return rec

    def end_group(comm, inst):
        """All ranks reached GroupEnd instance ``inst`` of ``comm``: move its
        messages, then run its allreduces in order, or fail the instance if a
        message is unmatched inside it or its allreduces disagree."""
        msgs = group_msgs.get((comm, inst), [])
        colls = group_colls.pop((comm, inst), {})
        ok = _colls_agree(colls, p.nranks)
        for key, k in msgs:
            c = chans[key]
            s, r = c.sends.get(k), c.recvs.get(k)
            if s is None or r is None or s.group != (comm, inst) or r.group != (comm, inst):
                ok = False
        if ok:
            for key, k in sorted(set(msgs)):
                if not chans[key].sends[k].done:
                    transfer(key, k)
            for i in range(len(colls.get(0, []))):
                reduce_instance({q: colls[q][i] for q in range(p.nranks)})
        group_ok[(comm, inst)] = ok
        for fn in group_after.pop((comm, inst), []):
            fn(ok)

    def reduce_instance(inst):
        """One allreduce over every rank: inst[q] is rank q's call."""
        op = inst[0]
        ins = []
        for q in range(p.nranks):
            a = inst[q]
            src = a.recvbuf if a.sendbuf == IN_PLACE else a.sendbuf
            off = a.roff if a.sendbuf == IN_PLACE else a.soff
            n = a.count * red.NP_DTYPE[a.dtype]().itemsize
            ins.append(bufs[q][src][off: off + n])
        out = red.allreduce_bytes(op.op, op.dtype, op.count, ins)
        for q in range(p.nranks):
            a = inst[q]
            bufs[q][a.recvbuf][a.roff: a.roff + out.size] = out

    def arrive(rank, op: Allreduce):
        k = coll_next.get((op.comm, rank), 0)
        coll_next[(op.comm, rank)] = k + 1
        inst = coll.setdefault((op.comm, k), {})
        inst[rank] = op
        if len(inst) == p.nranks:
            reduce_instance(inst)
            coll_done[(op.comm, k)] = True
        return (op.comm, k)

    def step(ctx: _Context) -> bool:
        """Advance one op of ``ctx``; False when it is blocked."""
        rank = ctx.rank
        op = ctx.ops[ctx.pc]
        if ctx.pending is not None:
            kind, obj = ctx.pending
            if kind == "init":
                if obj not in batch_ok:
                    return False
                if not batch_ok[obj]:
                    sync_errors[rank].append((ctx.thread, ctx.pc, "ERR_ARG"))
                ctx.pending = None
                ctx.pc += 1
                return True
            if kind == "group":
                if obj not in group_ok:
                    return False
                if not group_ok[obj]:
                    sync_errors[rank].append((ctx.thread, ctx.pc, "ERR_ARG"))
                ctx.pending = None
                ctx.pc += 1
                return True
            if kind == "coll":
                if not coll_done.get(obj, False):
                    return False
            elif kind == "waitall":
                if not all(rec.done for rec in obj):
                    return False
                for (name, st), rec in zip(op_status_pairs(op), obj):
                    if isinstance(rec, _RecvRec) and st is not None:
                        statuses[rank][st] = rec.status
                    requests[rank].pop(name, None)
            else:
                if not obj.done:
                    return False
                if isinstance(obj, _RecvRec) and op.status is not None:
                    statuses[rank][op.status] = obj.status
            ctx.pending = None
            ctx.pc += 1
            return True

        if isinstance(op, (Send, Recv)):
            err = _check_p2p(p, rank, op)
            if err:
                sync_errors[rank].append((ctx.thread, ctx.pc, err))
                ctx.pc += 1
                return True
            grp = group_open.get((rank, op.comm))
            if grp is not None and isinstance(op, Recv) and (op.source == ANY_SOURCE
                                                             or op.tag == ANY_TAG):
                err = "ERR_RANK" if op.source == ANY_SOURCE else "ERR_TAG"
                sync_errors[rank].append((ctx.thread, ctx.pc, err))
                ctx.pc += 1
                return True
            if grp is None and (p.matching == "queue" or p.multiplex(op.comm)):
                rec = post_send_q(rank, op) if isinstance(op, Send) else post_recv_q(rank, op)
                if op.req is not None:
                    requests[rank][op.req] = (rec, p.stream_of_op(rank, op))
                    ctx.pc += 1
                    return True
                ctx.pending = ("one", rec)
                return step(ctx)
            bname = persist_open.get((rank, op.comm))
            if bname is not None:
                batch_ops.setdefault((rank, bname), []).append(op)
                if op.req is not None:
                    requests[rank][op.req] = (("batch", bname), p.stream_of(rank, op.comm))
                ctx.pc += 1
                return True
            if grp is not None:
                record_grouped(rank, op, grp)
                ctx.pc += 1
                return True
            rec = (post_send(rank, op, grp) if isinstance(op, Send) else post_recv(rank, op, grp))
            if op.req is not None:
                requests[rank][op.req] = (rec, p.stream_of(rank, op.comm))
                ctx.pc += 1
                return True
            ctx.pending = ("one", rec)
            return step(ctx)
        if isinstance(op, Wait):
            if any(n not in requests[rank] for n in op.reqs):
                sync_errors[rank].append((ctx.thread, ctx.pc, "ERR_REQUEST"))
                ctx.pc += 1
                return True
            if len({requests[rank][n][1] for n in op.reqs}) > 1:
                sync_errors[rank].append((ctx.thread, ctx.pc, "ERR_STREAM"))
                ctx.pc += 1
                return True
            recs = [requests[rank][n][0] for n in op.reqs]
            recorded = [r for r in recs if isinstance(r, tuple)]
            if recorded:
                # waits on requests of an open persistent group are recorded too
                names = {r[1] for r in recorded}
                if len(recorded) != len(recs) or len(names) != 1:
                    raise ValueError("a wait mixes requests of a persistent group with others")
                bname = names.pop()
                if any(k[0] == rank and v == bname for k, v in persist_open.items()):
                    batch_ops.setdefault((rank, bname), []).append(op)
                # (after a failed GroupInit the wait only releases the requests)
                for n in op.reqs:
                    requests[rank].pop(n)
                ctx.pc += 1
                return True
            open_groups = [r.group for r in recs if r.group is not None and r.group not in group_ok]
            if open_groups:
                # inside its group: the statuses arrive at the group's end
                record_grouped(rank, op, recs[0].group)
                ctx.pc += 1
                return True
            ctx.pending = ("waitall", recs)
            return step(ctx)
        if isinstance(op, Allreduce):
            err = _check_allreduce(p, rank, op)
            if err:
                sync_errors[rank].append((ctx.thread, ctx.pc, err))
                ctx.pc += 1
                return True
            grp = group_open.get((rank, op.comm))
            if grp is not None:
                # grouped: runs at the group's end (or every start of a
                # persistent group), after the group's messages
                bname = persist_open.get((rank, op.comm))
                if bname is not None:
                    batch_ops.setdefault((rank, bname), []).append(op)
                else:
                    record_grouped(rank, op, grp)
                ctx.pc += 1
                return True
            ctx.pending = ("coll", arrive(rank, op))
            return step(ctx)
        if isinstance(op, User):
            _apply_user(bufs[rank], op.fn)
            ctx.pc += 1
            return True
        if isinstance(op, GroupStart):
            if not (0 <= op.comm < p.ncomms) or p.stream_of(rank, op.comm) is None:
                sync_errors[rank].append((ctx.thread, ctx.pc, "ERR_COMM"))
            elif (rank, op.comm) in group_open:
                sync_errors[rank].append((ctx.thread, ctx.pc, "ERR_ARG"))
            else:
                inst = group_next.get((rank, op.comm), 0)
                group_open[(rank, op.comm)] = (op.comm, inst)
                end = ctx.ends.get(ctx.pc)
                if isinstance(end, GroupInit):
                    persist_open[(rank, op.comm)] = end.batch
                    batch_ops.setdefault((rank, end.batch), [])
            ctx.pc += 1
            return True
        if isinstance(op, GroupInit):
            grp = group_open.get((rank, op.comm))
            if grp is None or persist_open.get((rank, op.comm)) != op.batch:
                sync_errors[rank].append((ctx.thread, ctx.pc, "ERR_ARG"))
                ctx.pc += 1
                return True
            del group_open[(rank, op.comm)]
            del persist_open[(rank, op.comm)]
            group_next[(rank, op.comm)] = grp[1] + 1
            if any(isinstance(v[0], tuple) and v[0] == ("batch", op.batch)
                   for v in requests[rank].values()):
                batch_bad[op.batch] = True     # a request of the group is never waited for
            arrived = batch_arrived.setdefault(op.batch, set())
            arrived.add(rank)
            if len(arrived) == p.nranks:
                init_batch(op.batch)
            ctx.pending = ("init", op.batch)
            return step(ctx)
        if isinstance(op, Start):
            if not batch_ok.get(op.batch, False):
                sync_errors[rank].append((ctx.thread, ctx.pc, "ERR_REQUEST"))
                ctx.pc += 1
                return True
            j = batch_runs.get((rank, op.batch), 0)
            batch_runs[(rank, op.batch)] = j + 1
            grp = (("batch", op.batch), j)
            for o in batch_ops[(rank, op.batch)]:
                record_grouped(rank, o, grp)
            arrived = group_arrived.setdefault(grp, set())
            arrived.add(rank)
            if len(arrived) == p.nranks:
                end_group(*grp)
            ctx.pending = ("group", grp)
            return step(ctx)
        if isinstance(op, GroupEnd):
            grp = group_open.pop((rank, op.comm), None)
            if grp is None:
                sync_errors[rank].append((ctx.thread, ctx.pc, "ERR_ARG"))
                ctx.pc += 1
                return True
            group_next[(rank, op.comm)] = grp[1] + 1
            arrived = group_arrived.setdefault(grp, set())
            arrived.add(rank)
            if len(arrived) == p.nranks:
                end_group(*grp)
            ctx.pending = ("group", grp)
            return step(ctx)
        raise ValueError(f"unknown op {op!r}")

    def op_status_pairs(op: Wait):
        return list(zip(op.reqs, op.statuses))

    ctxs = [_Context(r, t, p.ops[r][t]) for r in range(p.nranks)
            for t in range(len(p.ops[r]))]
    for c in ctxs:
        c.ends = terminators(c.ops)
    deadlock = False
    for _ in range(max_rounds):
        progressed = False
        for ctx in ctxs:
            while ctx.pc < len(ctx.ops) and step(ctx):
                progressed = True
        if all(c.pc >= len(c.ops) for c in ctxs):
            break
        if not progressed:
            deadlock = True
            break
    blocked = [(c.rank, c.thread, c.pc) for c in ctxs if c.pc < len(c.ops)]
    return Result(bufs, statuses, sync_errors, match_log, deadlock, blocked)
