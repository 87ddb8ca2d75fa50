"""Program descriptions shared by the oracle and the GPU runner.

A *program* is what N rank threads do: each rank owns some byte buffers and an
ordered list of operations.  Operations name buffers by string and give byte
offsets into them; datatypes are given as constructor trees::

    "int32"                                  a basic type
    ("contiguous", n, T)
    ("vector", count, blocklength, stride, T)
    ("indexed", [blocklengths], [displacements], T)

Threads and streams: rank ``r`` has ``streams_per_rank`` streams (each maps to
one HIP stream on the GPU path) and ``len(ops[r])`` host threads; thread ``t``
runs the op list ``ops[r][t]`` in order.  Communicator ``c`` spans all ranks;
on rank ``r`` it is attached to stream ``comm_streams[c][r]`` (``None``: the
rank built the communicator with a null stream, so enqueue calls on it are
erroneous).  A stream is driven by one thread only, which is the
serial-context contract of the stream object; one thread may drive several
streams.

Nothing here computes a result of the method.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Union

import numpy as np

#: basic datatypes and their sizes in bytes
BASIC_TYPES = {
    "uint8": 1, "int8": 1,
    "int32": 4, "float32": 4,
    "int64": 8, "float64": 8,
}

#: special argument values (as in MPI, wildcards are negative)
ANY_SOURCE = -2
ANY_INDEX = -3
ANY_TAG = -1
IN_PLACE = "__in_place__"

TypeTree = Union[str, tuple]


@dataclass
class Send:
    """send (blocking) or isend (``req`` names the request)."""
    buf: str
    off: int
    count: int
    dtype: TypeTree
    dest: int
    tag: int
    comm: int = 0
    req: Optional[str] = None        # set => isend
    # multiplex communicators: stream indices (src_idx is this rank's)
    src_idx: Optional[int] = None
    dst_idx: Optional[int] = None

    @property
    def kind(self):
        return "isend" if self.req is not None else "send"


@dataclass
class Recv:
    """recv (blocking, ``status`` names a status slot or None) or irecv."""
    buf: str
    off: int
    count: int
    dtype: TypeTree
    source: int
    tag: int
    comm: int = 0
    req: Optional[str] = None        # set => irecv
    status: Optional[str] = None
    # multiplex communicators: stream indices (dst_idx is this rank's;
    # src_idx may be ANY_INDEX)
    src_idx: Optional[int] = None
    dst_idx: Optional[int] = None

    @property
    def kind(self):
        return "irecv" if self.req is not None else "recv"


@dataclass
class Wait:
    """wait (one request) or waitall (several); statuses may be None."""
    reqs: List[str]
    statuses: List[Optional[str]]

    @property
    def kind(self):
        return "wait" if len(self.reqs) == 1 else "waitall"


@dataclass
class Allreduce:
    sendbuf: str                     # buffer name or IN_PLACE
    soff: int
    recvbuf: str
    roff: int
    count: int
    dtype: str                       # basic type name
    op: str                          # "sum" | "prod" | "min" | "max"
    comm: int = 0

    kind = "allreduce"


@dataclass
class User:
    """A deterministic user kernel placed on the rank's stream.

    fn is one of
      ("add_const_i32", buf, off, n, c)            x[i] += c        (int32, wraps)
      ("saxpy_f32", xbuf, xoff, ybuf, yoff, n, a)  y[i] = a*x[i] + y[i]
      ("add_rows_f32", dst, doff, src, soff, rows, row_elems, col_lo, col_hi)
                       dst[r, c] += src[r, c] for c in [col_lo, col_hi)
    ``stream`` is the rank's stream it is launched on.
    """
    fn: tuple
    stream: int = 0

    kind = "user"


@dataclass
class GroupStart:
    """Start recording this rank's operations on ``comm`` (a batch)."""
    comm: int = 0

    kind = "group_start"


@dataclass
class GroupEnd:
    """Collective end of the rank's current group on ``comm``."""
    comm: int = 0

    kind = "group_end"


@dataclass
class GroupInit:
    """Collective end of the rank's current group on ``comm`` that keeps the
    group as the persistent batch ``batch`` instead of running it."""
    batch: str
    comm: int = 0

    kind = "group_init"


@dataclass
class Start:
    """One run of the persistent batch ``batch`` (made on ``comm``)."""
    batch: str
    comm: int = 0

    kind = "start"


Op = Union[Send, Recv, Wait, Allreduce, User, GroupStart, GroupEnd, GroupInit, Start]


@dataclass
class Program:
    nranks: int
    buffers: List[Dict[str, np.ndarray]]           # per rank: name -> uint8 array
    ops: List[List[List[Op]]]                      # ops[rank][thread]
    streams_per_rank: int = 1
    comm_streams: List[List[Optional[int]]] = field(default_factory=list)
    name: str = ""
    # "sequence": k-th send meets k-th receive per (comm, src, dst, tag), no
    # wildcards; "queue": ordered posted / unexpected queues per destination,
    # receives may use ANY_SOURCE / ANY_TAG
    matching: str = "sequence"

    def __post_init__(self):
        if not self.comm_streams:
            self.comm_streams = [[0] * self.nranks]
        if len(self.ops) != self.nranks or len(self.buffers) != self.nranks:
            raise ValueError("one op table and one buffer set per rank")
        for r in range(self.nranks):
            owner = {}
            req_thread = {}
            for t, lst in enumerate(self.ops[r]):
                for o in lst:
                    name = getattr(o, "req", None)
                    if name is not None and req_thread.setdefault(name, t) != t:
                        raise ValueError(f"rank {r}: request {name!r} used by two threads")
                    st = self.stream_of_op(r, o)
                    if st is None:
                        continue
                    if not 0 <= st < self.streams_per_rank:
                        raise ValueError(f"rank {r}: stream {st} out of range")
                    if owner.setdefault(st, t) != t:
                        raise ValueError(f"rank {r}: stream {st} driven by two threads")
        for r, bufs in enumerate(self.buffers):
            for k, v in bufs.items():
                if v.dtype != np.uint8 or v.ndim != 1:
                    raise ValueError(f"rank {r} buffer {k}: want flat uint8")

    @property
    def ncomms(self):
        return len(self.comm_streams)

    def multiplex(self, comm: int) -> bool:
        """A multiplex communicator lists several streams per rank."""
        return any(isinstance(x, list) for x in self.comm_streams[comm])

    def stream_of(self, rank: int, comm: int) -> Optional[int]:
        """The rank's single stream of a communicator (None for none, and for
        multiplex communicators, which have no single stream)."""
        x = self.comm_streams[comm][rank]
        return None if isinstance(x, list) else x

    def stream_of_op(self, rank: int, o) -> Optional[int]:
        """The stream an operation of ``rank`` runs on, if any."""
        if isinstance(o, User):
            return o.stream
        c = getattr(o, "comm", None)
        if c is None or not (0 <= c < len(self.comm_streams)):
            return None
        x = self.comm_streams[c][rank]
        if isinstance(x, list):
            local = getattr(o, "src_idx" if isinstance(o, Send) else "dst_idx", None)
            return x[local] if isinstance(local, int) and 0 <= local < len(x) else None
        return x

    def copy_buffers(self) -> List[Dict[str, np.ndarray]]:
        return [{k: v.copy() for k, v in b.items()} for b in self.buffers]


def as_bytes(a: np.ndarray) -> np.ndarray:
    """View any contiguous numpy array as a flat uint8 array (a copy)."""
    return np.ascontiguousarray(a).view(np.uint8).reshape(-1).copy()


def footprint_bound(tree: TypeTree, count: int) -> int:
    """A generous upper bound on the bytes ``count`` elements of ``tree`` can
    reach from their start address, used only to lay out test buffers.

    It over-counts on purpose (every block is charged max(stride, blocklength)
    old-type bounds), so it never has to agree with a datatype's true extent.
    """
    def one(t) -> int:
        if isinstance(t, str):
            return BASIC_TYPES[t]
        if t[0] == "contiguous":
            return t[1] * one(t[2])
        if t[0] == "vector":
            return t[1] * max(t[2], t[3]) * one(t[4])
        if t[0] == "indexed":
            reach = max([d + b for b, d in zip(t[1], t[2])], default=0)
            return reach * one(t[3])
        raise ValueError(t)
    return max(count, 0) * one(tree)


def count_messages(p: Program) -> int:
    return sum(1 for per_rank in p.ops for ops in per_rank for o in ops
               if isinstance(o, Send))


def single_stream(nranks, buffers, ops, name="", ncomms=1) -> Program:
    """A program whose ranks each drive one stream (op lists given per rank)."""
    return Program(nranks=nranks, buffers=buffers, ops=[[o] for o in ops],
                   streams_per_rank=1, comm_streams=[[0] * nranks for _ in range(ncomms)],
                   name=name)


def streams_of_thread(p: Program, rank: int, thread: int) -> List[int]:
    """Streams that thread ``thread`` of ``rank`` drives (in first-use order)."""
    out = []
    for o in p.ops[rank][thread]:
        st = p.stream_of_op(rank, o)
        if st is not None and st not in out:
            out.append(st)
    return out


Tree = TypeTree
__all__ = [
    "Program", "Send", "Recv", "Wait", "Allreduce", "User", "GroupStart", "GroupEnd",
    "GroupInit", "Start", "IN_PLACE",
    "ANY_SOURCE", "ANY_TAG", "ANY_INDEX", "BASIC_TYPES", "as_bytes", "count_messages", "Tree",
    "single_stream", "footprint_bound", "streams_of_thread",
]
