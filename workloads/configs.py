"""Seeded synthetic programs for the benchmark configurations and the tests.

Every random draw uses ``numpy.random.default_rng([220813707, config, rank,
step])`` (PCG64), so the oracle and the GPU path see the same bytes.  Nothing
here computes a result of the method: these functions only lay out buffers
and the operations each rank issues.

Configurations (one MI355X; ranks are host threads):
  1  ping-pong: 2 ranks, 1000 blocking messages of 1024 int32 (uniform over
     the full int32 range), tag 0, one communicator.
  2  ring halo: 8 ranks; per rank A, H float32[count * 8] ~ N(0, 1);
     datatype vector(count, 3, 8, float32); per step s (tag s) each rank
     isends columns 0..2 of A to its right neighbour and columns 3..5 to its
     left neighbour and receives them into H; count in {2730, 5461, 10922,
     21845, 43690} (payload 32,760 .. 524,280 bytes).
  3  allreduce: 16 ranks, SUM on int64 (uniform in [-2^40, 2^40]) and float32
     (~ N(0, 1)), 4 KiB, 1 MiB and 64 MiB per rank.
  4  batch: 32 ranks, 10,000 send/recv pairs, bytes log-uniform in
     [8, 262144], tags uniform in 0..63, 30 % vector datatypes.
"""
from __future__ import annotations

import math
from typing import List, Optional

import numpy as np

from .program import (
    ANY_SOURCE, ANY_TAG, IN_PLACE, Allreduce, GroupEnd, GroupInit, GroupStart, Program, Recv,
    Send, Start, User, Wait, as_bytes, footprint_bound, single_stream,
)

SEED = 220813707

HALO_COUNTS = (2730, 5461, 10922, 21845, 43690)
ALLREDUCE_BYTES = (4 * 1024, 1024 * 1024, 64 * 1024 * 1024)


def rng(config: int, rank: int = 0, step: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED, config, rank, step])


# --------------------------------------------------------------------------- 1
def pingpong(nmsg: int = 1000, n: int = 1024, increment: bool = False,
             seed_config: int = 1) -> Program:
    """Config 1: rank 0 sends x to rank 1 and receives it back; rank 1 does
    the reverse.  With ``increment`` rank 1 adds 1 to every element between
    its receive and its send (a user kernel on its stream)."""
    assert nmsg % 2 == 0
    x0 = rng(seed_config, 0).integers(-2**31, 2**31, size=n, dtype=np.int64).astype(np.int32)
    bufs = [{"x": as_bytes(x0)}, {"x": np.zeros(4 * n, dtype=np.uint8)}]
    r0, r1 = [], []
    for _ in range(nmsg // 2):
        r0 += [Send("x", 0, n, "int32", 1, 0), Recv("x", 0, n, "int32", 1, 0)]
        r1 += [Recv("x", 0, n, "int32", 0, 0)]
        if increment:
            r1 += [User(("add_const_i32", "x", 0, n, 1))]
        r1 += [Send("x", 0, n, "int32", 0, 0)]
    return single_stream(2, bufs, [r0, r1], name=f"pingpong_{nmsg}x{n}")


# --------------------------------------------------------------------------- 2
def halo_type(count: int):
    return ("vector", count, 3, 8, "float32")


def ring_halo(count: int = 2730, steps: int = 100, nranks: int = 8,
              update: bool = False, blocking_recv: bool = True, grouped: bool = False,
              persistent: bool = False) -> Program:
    """Config 2: bidirectional ring halo exchange with a vector datatype.
    ``grouped``: each step's operations form one group (one batch).
    ``persistent``: one step's operations (tag 0) are recorded once as the
    persistent batch "halo", which every step starts."""
    if persistent:
        return _ring_halo_persistent(count, steps, nranks, update, blocking_recv)
    vt = halo_type(count)
    bufs, ops = [], []
    for r in range(nranks):
        g = rng(2, r)
        a = g.standard_normal(count * 8, dtype=np.float32)
        h = g.standard_normal(count * 8, dtype=np.float32)
        bufs.append({"A": as_bytes(a), "H": as_bytes(h)})
        right, left = (r + 1) % nranks, (r - 1) % nranks
        lst = []
        for s in range(steps):
            if grouped:
                lst.append(GroupStart())
            lst += [Send("A", 0, 1, vt, right, s, req=f"s{s}a"),
                    Send("A", 12, 1, vt, left, s, req=f"s{s}b")]
            if blocking_recv:
                lst += [Recv("H", 0, 1, vt, left, s, status=f"st{s}a"),
                        Recv("H", 12, 1, vt, right, s, status=f"st{s}b")]
                lst += [Wait([f"s{s}a", f"s{s}b"], [None, None])]
            else:
                lst += [Recv("H", 0, 1, vt, left, s, req=f"r{s}a"),
                        Recv("H", 12, 1, vt, right, s, req=f"r{s}b")]
                lst += [Wait([f"s{s}a", f"s{s}b", f"r{s}a", f"r{s}b"],
                             [None, None, f"st{s}a", f"st{s}b"])]
            if grouped:
                lst.append(GroupEnd())
            if update:
                lst += [User(("add_rows_f32", "A", 0, "H", 0, count, 8, 0, 6))]
        ops.append(lst)
    return single_stream(nranks, bufs, ops,
                         name=f"ring_halo_{nranks}r_c{count}_s{steps}" + ("_grouped" if grouped else ""))


def _ring_halo_persistent(count, steps, nranks, update, blocking_recv) -> Program:
    vt = halo_type(count)
    bufs, ops = [], []
    for r in range(nranks):
        g = rng(2, r)
        a = g.standard_normal(count * 8, dtype=np.float32)
        h = g.standard_normal(count * 8, dtype=np.float32)
        bufs.append({"A": as_bytes(a), "H": as_bytes(h)})
        right, left = (r + 1) % nranks, (r - 1) % nranks
        lst = [GroupStart(), Send("A", 0, 1, vt, right, 0, req="sa"),
               Send("A", 12, 1, vt, left, 0, req="sb")]
        if blocking_recv:
            lst += [Recv("H", 0, 1, vt, left, 0, status="sta"),
                    Recv("H", 12, 1, vt, right, 0, status="stb"),
                    Wait(["sa", "sb"], [None, None])]
        else:
            lst += [Recv("H", 0, 1, vt, left, 0, req="ra"),
                    Recv("H", 12, 1, vt, right, 0, req="rb"),
                    Wait(["sa", "sb", "ra", "rb"], [None, None, "sta", "stb"])]
        lst.append(GroupInit("halo"))
        for _ in range(steps):
            lst.append(Start("halo"))
            if update:
                lst.append(User(("add_rows_f32", "A", 0, "H", 0, count, 8, 0, 6)))
        ops.append(lst)
    return single_stream(nranks, bufs, ops,
                         name=f"ring_halo_{nranks}r_c{count}_s{steps}_persistent")


# --------------------------------------------------------------------------- 3
def allreduce(nbytes: int, dtype: str = "int64", nranks: int = 16, calls: int = 1,
              op: str = "sum", in_place: bool = False) -> Program:
    """Config 3: ``calls`` allreduces of ``nbytes`` per rank."""
    esize = {"int32": 4, "int64": 8, "float32": 4, "float64": 8}[dtype]
    count = nbytes // esize
    bufs, ops = [], []
    for r in range(nranks):
        g = rng(3, r)
        if dtype in ("int64", "int32"):
            lim = 2**40 if dtype == "int64" else 2**30
            x = g.integers(-lim, lim + 1, size=count, dtype=np.int64).astype(dtype)
        else:
            x = g.standard_normal(count).astype(dtype)
        if in_place:
            bufs.append({"recv": as_bytes(x)})
            ops.append([Allreduce(IN_PLACE, 0, "recv", 0, count, dtype, op)
                        for _ in range(calls)])
        else:
            bufs.append({"send": as_bytes(x), "recv": np.zeros(nbytes, np.uint8)})
            ops.append([Allreduce("send", 0, "recv", 0, count, dtype, op)
                        for _ in range(calls)])
    return single_stream(nranks, bufs, ops, name=f"allreduce_{nranks}r_{dtype}_{nbytes}B")


# --------------------------------------------------------------------------- 4
def batch_messages(npairs: int = 10000, nranks: int = 32, max_bytes: int = 262144,
                   min_bytes: int = 8, vec_frac: float = 0.3, seed_config: int = 4):
    """Config 4 message list: (src, dst, tag, dtype tree, count, nbytes)."""
    g = rng(seed_config, 0)
    msgs = []
    for _ in range(npairs):
        src = int(g.integers(nranks))
        dst = int(g.integers(nranks - 1))
        dst = dst + 1 if dst >= src else dst
        tag = int(g.integers(64))
        nbytes = int(math.floor(math.exp(g.uniform(math.log(min_bytes), math.log(max_bytes)))))
        if g.uniform() < vec_frac:
            bl = int(g.integers(1, 17))
            base = "float32" if g.uniform() < 0.5 else "int32"
            c = max(1, -(-nbytes // (4 * bl)))
            tree = ("vector", c, bl, 2 * bl, base)
            size = 4 * bl * c
        else:
            base = ("uint8", "int32", "float32")[int(g.integers(3))]
            es = 1 if base == "uint8" else 4
            c = max(1, nbytes // es)
            tree = base
            size = c * es
        count = 1 if isinstance(tree, tuple) else c
        msgs.append(dict(src=src, dst=dst, tag=tag, tree=tree, count=count,
                         size=size, foot=footprint_bound(tree, count)))
    return msgs


def batch(npairs: int = 10000, nranks: int = 32, max_bytes: int = 262144,
          min_bytes: int = 8, grouped: bool = False, runs: int = 0) -> Program:
    """Config 4: every rank isends all its messages in global order, then
    irecvs all its messages in global order, then waits for all of them.
    ``grouped``: all of it is one group (one batch).  ``runs`` > 0: the
    group is recorded once as the persistent batch "batch" and started
    ``runs`` times; before every run but the first, each rank adds 1 to
    every int32 word of its send buffer, so each run moves new bytes."""
    msgs = batch_messages(npairs, nranks, max_bytes, min_bytes)
    send_off = [0] * nranks
    recv_off = [0] * nranks
    ops: List[list] = [[] for _ in range(nranks)]
    recvs: List[list] = [[] for _ in range(nranks)]
    align = 256
    for i, m in enumerate(msgs):
        s, d = m["src"], m["dst"]
        ops[s].append(Send("sbuf", send_off[s], m["count"], m["tree"], d, m["tag"], req=f"s{i}"))
        recvs[d].append(Recv("rbuf", recv_off[d], m["count"], m["tree"], s, m["tag"],
                             req=f"r{i}"))
        send_off[s] += -(-m["foot"] // align) * align
        recv_off[d] += -(-m["foot"] // align) * align
    bufs = []
    for r in range(nranks):
        g = rng(4, r, 1)
        sb = g.integers(0, 256, size=max(send_off[r], 1), dtype=np.uint8)
        rb = g.integers(0, 256, size=max(recv_off[r], 1), dtype=np.uint8)
        bufs.append({"sbuf": sb, "rbuf": rb})
        reqs = [o.req for o in ops[r]] + [o.req for o in recvs[r]]
        stats = [None] * len(ops[r]) + [f"st_{o.req}" for o in recvs[r]]
        ops[r] = ops[r] + recvs[r]
        if reqs:
            ops[r].append(Wait(reqs, stats))
        if runs > 0:
            body = [GroupStart()] + ops[r] + [GroupInit("batch")]
            for j in range(runs):
                if j:
                    body.append(User(("add_const_i32", "sbuf", 0, sb.size // 4, 1)))
                body.append(Start("batch"))
            ops[r] = body
        elif grouped:
            ops[r] = [GroupStart()] + ops[r] + [GroupEnd()]
    suffix = f"_persistent{runs}" if runs > 0 else ("_grouped" if grouped else "")
    return single_stream(nranks, bufs, ops, name=f"batch_{npairs}p_{nranks}r" + suffix)


# --------------------------------------------------------------------- 5
SERVE_KINDS = {"sendrecv": 0, "isend_wait": 1, "allreduce": 2}


def serving_schedule(rate: float, nreq: int, nranks: int = 64, min_bytes: int = 64,
                     max_bytes: int = 4 << 20, seed: int = 0):
    """Config 5: an open-loop Poisson stream of ``nreq`` requests at ``rate``
    per second: 60 % send/recv, 30 % isend+wait, 10 % allreduce-sum int32
    (over all ranks), bytes log-uniform in [min_bytes, max_bytes] (allreduce:
    per rank, a multiple of 4).  Returns a list of dicts sorted by arrival."""
    g = rng(5, seed)
    t = np.cumsum(g.exponential(1e6 / rate, size=nreq))
    out = []
    for i in range(nreq):
        u = g.uniform()
        kind = 0 if u < 0.6 else (1 if u < 0.9 else 2)
        nbytes = int(math.floor(math.exp(g.uniform(math.log(min_bytes), math.log(max_bytes)))))
        src = int(g.integers(nranks))
        dst = int(g.integers(nranks - 1))
        dst = dst + 1 if dst >= src else dst
        if kind == 2:
            nbytes = max(4, nbytes // 4 * 4)
            src = dst = 0
        out.append(dict(kind=kind, src=src, dst=dst, bytes=nbytes, arrival_us=float(t[i]),
                        seed=(seed << 24) + i + 1))
    return out


# ------------------------------------------------------------------- examples
def saxpy_example(n: int = 4096) -> Program:
    """The paper's GPU enqueue example (§6): rank 0 sends x (all 1.0) to rank
    1, which receives it and computes y = a*x + y with a = 2, y = 2."""
    x = np.full(n, 1.0, np.float32)
    y = np.full(n, 2.0, np.float32)
    bufs = [{"x": as_bytes(x)},
            {"x": np.zeros(4 * n, np.uint8), "y": as_bytes(y)}]
    r0 = [Send("x", 0, n, "float32", 1, 0)]
    r1 = [Recv("x", 0, n, "float32", 0, 0),
          User(("saxpy_f32", "x", 0, "y", 0, n, 2.0))]
    return single_stream(2, bufs, [r0, r1], name="saxpy")


def threads_example(nthreads: int = 4, n: int = 100) -> Program:
    """The paper's MPI+OpenMP example (§6): 2 ranks, each with ``nthreads``
    streams and one stream communicator per stream; context i of rank 0
    sends 100 chars to context i of rank 1."""
    bufs = []
    for r in range(2):
        g = rng(6, r)
        bufs.append({f"buf{i}": g.integers(0, 256, size=n, dtype=np.uint8)
                     for i in range(nthreads)})
    ops = [[[Send(f"buf{i}", 0, n, "uint8", 1, 0, comm=i)] for i in range(nthreads)],
           [[Recv(f"buf{i}", 0, n, "uint8", 0, 0, comm=i)] for i in range(nthreads)]]
    comm_streams = [[i, i] for i in range(nthreads)]
    return Program(nranks=2, buffers=bufs, ops=ops, streams_per_rank=nthreads,
                   comm_streams=comm_streams, name=f"threads_{nthreads}")


# --------------------------------------------------------------- random safe
def random_program(seed: int, nranks: int = 4, nmsg: int = 40, max_elems: int = 300,
                   tags: int = 3, ncomms: int = 2, allreduces: int = 2,
                   types: Optional[list] = None, grouped: bool = False) -> Program:
    """A random program that is safe under synchronous-send semantics.

    Messages are drawn as (src, dst, comm, tag, datatype); each rank issues
    its isends in message order, then its irecvs in message order, then
    waits for all.  Allreduces are placed after the waits.  Send buffers are
    read-only; every receive gets its own region of the receive buffer, and
    the gaps between regions keep their initial bytes.
    """
    g = np.random.default_rng([SEED, 100, seed])
    if types is None:
        types = [
            lambda n: ("int32", n),
            lambda n: ("float32", n),
            lambda n: ("uint8", n * 4),
            lambda n: (("vector", max(1, n // 3), 3, 5, "int32"), 1),
            lambda n: (("vector", max(1, n // 2), 2, 7, "float64"), 1),
            lambda n: (("contiguous", 2, ("vector", max(1, n // 4), 1, 3, "int32")), 2),
            lambda n: (("indexed", [3, 1, 4, 2], [0, 5, 7, 13], "int32"), max(1, n // 10)),
            lambda n: (("vector", 2, 2, 3, ("indexed", [1, 2], [4, 0], "int64")), max(1, n // 12)),
        ]
    msgs = []
    for i in range(nmsg):
        s = int(g.integers(nranks))
        d = int(g.integers(nranks))
        if nranks > 1 and d == s and g.uniform() < 0.8:
            d = (s + 1 + int(g.integers(nranks - 1))) % nranks
        comm = int(g.integers(ncomms))
        tag = int(g.integers(tags))
        n = int(g.integers(0, max_elems + 1))
        tree, cnt = types[int(g.integers(len(types)))](n)
        msgs.append((s, d, comm, tag, tree, cnt))
    send_off = [0] * nranks
    recv_off = [0] * nranks
    sends: List[list] = [[] for _ in range(nranks)]
    recvs: List[list] = [[] for _ in range(nranks)]
    for i, (s, d, comm, tag, tree, cnt) in enumerate(msgs):
        foot = footprint_bound(tree, cnt)
        sends[s].append(Send("sbuf", send_off[s], cnt, tree, d, tag, comm=comm, req=f"s{i}"))
        recvs[d].append(Recv("rbuf", recv_off[d], cnt, tree, s, tag, comm=comm, req=f"r{i}"))
        send_off[s] += foot + int(g.integers(0, 3)) * 8
        recv_off[d] += foot + 16
    bufs, ops = [], []
    for r in range(nranks):
        gr = np.random.default_rng([SEED, 100, seed, r])
        red_n = 64
        b = {"sbuf": gr.integers(0, 256, size=send_off[r] + 64, dtype=np.uint8),
             "rbuf": gr.integers(0, 256, size=recv_off[r] + 64, dtype=np.uint8),
             "ared": as_bytes(gr.integers(-2**40, 2**40, size=red_n, dtype=np.int64)),
             "afl": as_bytes(gr.standard_normal(red_n).astype(np.float32)),
             "aout": np.zeros(8 * red_n, np.uint8)}
        bufs.append(b)
        lst = sends[r] + recvs[r]
        reqs = [o.req for o in lst]
        if reqs:
            lst = list(lst)
            lst.append(Wait(reqs, [f"st_{q}" if q.startswith("r") else None for q in reqs]))
        if grouped:
            # one group per communicator (all on the rank's single stream)
            lst = ([GroupStart(c) for c in range(ncomms)] + lst
                   + [GroupEnd(c) for c in range(ncomms)])
        for a in range(allreduces):
            if a % 2 == 0:
                lst.append(Allreduce("ared", 0, "aout", 0, red_n, "int64", "sum"))
            else:
                lst.append(Allreduce("afl", 0, "aout", 0, red_n, "float32", "sum"))
        ops.append(lst)
    return Program(nranks=nranks, buffers=bufs, ops=[[o] for o in ops], streams_per_rank=1,
                   comm_streams=[[0] * nranks for _ in range(ncomms)],
                   name=f"random_{seed}" + ("_grouped" if grouped else ""))


# ------------------------------------------------------------------ wildcards
def _queue(nranks, bufs, ops, name="wild") -> Program:
    p = single_stream(nranks, bufs, ops, name=name)
    p.matching = "queue"
    return p


def wildcard_programs():
    """Programs whose wildcard matches are the same in every interleaving."""
    out = []
    # ANY_TAG from one sender: messages arrive in send order (non-overtaking)
    b = [{"s": as_bytes(np.array([50, 30, 70], np.int32))}, {"r": np.zeros(12, np.uint8)}]
    ops = [[Send("s", 4 * i, 1, "int32", 1, t) for i, t in enumerate((5, 3, 7))],
           [Recv("r", 4 * i, 1, "int32", 0, ANY_TAG, status=f"st{i}") for i in range(3)]]
    out.append(_queue(2, b, ops, "any-tag-in-order"))
    # ANY_SOURCE told apart by tags
    b = [{"s": as_bytes(np.array([100 + q], np.int32)), "r": np.zeros(8, np.uint8)}
         for q in range(3)]
    ops = [[Send("s", 0, 1, "int32", 1, 10)],
           [Recv("r", 0, 1, "int32", ANY_SOURCE, 20, status="a"),
            Recv("r", 4, 1, "int32", ANY_SOURCE, 10, status="b")],
           [Send("s", 0, 1, "int32", 1, 20)]]
    out.append(_queue(3, b, ops, "any-source-by-tag"))
    # a wildcard receive posted before a specific one takes the first message
    b = [{"s": as_bytes(np.array([1, 2], np.int32))}, {"r": np.zeros(8, np.uint8)}]
    ops = [[Send("s", 0, 1, "int32", 1, 4, req="x"), Send("s", 4, 1, "int32", 1, 4, req="y"),
            Wait(["x", "y"], [None, None])],
           [Recv("r", 0, 1, "int32", ANY_SOURCE, ANY_TAG, req="w", status=None),
            Recv("r", 4, 1, "int32", 0, 4, req="v"), Wait(["w", "v"], ["sw", "sv"])]]
    out.append(_queue(2, b, ops, "posted-order"))
    return out


def competing_senders(nsend=3, per=4):
    """Ranks 1..nsend each send `per` messages (value 1000 * src + i) to rank
    0, which receives them all with ANY_SOURCE / ANY_TAG."""
    n = nsend + 1
    bufs = [{"r": np.zeros(4 * nsend * per, np.uint8)}]
    ops = [[Recv("r", 4 * j, 1, "int32", ANY_SOURCE, ANY_TAG, status=f"s{j}")
            for j in range(nsend * per)]]
    for q in range(1, n):
        bufs.append({"s": as_bytes(np.array([1000 * q + i for i in range(per)], np.int32))})
        ops.append([Send("s", 4 * i, 1, "int32", 0, 7 + i) for i in range(per)])
    return _queue(n, bufs, ops, "competing")


# ------------------------------------------------------------ multiplex (§3.5)
def multiplex_n_to_1(nthreads: int = 4, per: int = 3, racing: bool = False) -> Program:
    """The paper's N-to-1 use of a multiplex stream communicator: rank 0 runs
    ``nthreads`` threads, each on its own stream (index i), isending ``per``
    messages (value 100 * i + j, tag 10 * i + j) to the single polling
    thread of rank 1 (index 0), which receives them all on one communicator
    with ANY_INDEX -- by tag, in reverse order (each match unique), or with
    ANY_TAG as well (``racing``: the senders race)."""
    from .program import ANY_INDEX
    bufs = [{"s": as_bytes(np.array([100 * i + j for i in range(nthreads) for j in range(per)],
                                    np.int32))},
            {"r": np.zeros(4 * nthreads * per, np.uint8)}]
    # request names are per rank: each thread uses its own
    senders = [[Send("s", 4 * (i * per + j), 1, "int32", 1, 10 * i + j, req=f"m{i}_{j}",
                     src_idx=i, dst_idx=0) for j in range(per)]
               + [Wait([f"m{i}_{j}" for j in range(per)], [None] * per)] for i in range(nthreads)]
    order = [(i, j) for i in range(nthreads) for j in range(per)]
    if racing:
        recv = [Recv("r", 4 * k, 1, "int32", 0, ANY_TAG, status=f"s{k}", src_idx=ANY_INDEX,
                     dst_idx=0) for k in range(len(order))]
    else:
        recv = [Recv("r", 4 * k, 1, "int32", 0, 10 * i + j, status=f"s{k}", src_idx=ANY_INDEX,
                     dst_idx=0) for k, (i, j) in enumerate(reversed(order))]
    return Program(nranks=2, buffers=bufs, ops=[senders, [recv]], streams_per_rank=nthreads,
                   comm_streams=[[list(range(nthreads)), [0]]],
                   name=f"multiplex_{nthreads}to1" + ("_racing" if racing else ""))


def multiplex_all_pairs(nthreads: int = 2) -> Program:
    """Two ranks with ``nthreads`` streams each on one multiplex communicator:
    thread i of each rank sends one message to every thread j of the other
    rank (indices i -> j, value 1000 * rank + 10 * i + j) and receives one
    from every thread of the other rank, addressed by index."""
    bufs, ops = [], []
    for r in range(2):
        vals = [1000 * r + 10 * i + j for i in range(nthreads) for j in range(nthreads)]
        bufs.append({"s": as_bytes(np.array(vals, np.int32)),
                     "r": np.zeros(4 * nthreads * nthreads, np.uint8)})
        threads = []
        for i in range(nthreads):
            lst = [Send("s", 4 * (i * nthreads + j), 1, "int32", 1 - r, 5, req=f"x{i}_{j}",
                        src_idx=i, dst_idx=j) for j in range(nthreads)]
            lst += [Recv("r", 4 * (i * nthreads + j), 1, "int32", 1 - r, 5, req=f"y{i}_{j}",
                         src_idx=j, dst_idx=i) for j in range(nthreads)]
            lst.append(Wait([f"x{i}_{j}" for j in range(nthreads)]
                            + [f"y{i}_{j}" for j in range(nthreads)],
                            [None] * nthreads + [f"st{i}_{j}" for j in range(nthreads)]))
            threads.append(lst)
        ops.append(threads)
    return Program(nranks=2, buffers=bufs, ops=ops, streams_per_rank=nthreads,
                   comm_streams=[[list(range(nthreads)), list(range(nthreads))]],
                   name=f"multiplex_pairs_{nthreads}")


# ------------------------------------------------------------- degenerate
def degenerate_programs():
    """Degenerate cases: a one-rank world (messages to itself, an allreduce
    over one rank, a zero-count allreduce), and two ranks with an empty
    one-shot group, a zero-count allreduce, and an empty persistent group
    started twice."""
    out = []
    b = [{"a": as_bytes(np.arange(1, 6, dtype=np.int32)), "b": np.zeros(20, np.uint8),
          "c": np.zeros(20, np.uint8)}]
    ops = [[Send("a", 0, 5, "int32", 0, 7, req="s"), Recv("b", 0, 5, "int32", 0, 7, status="st"),
            Wait(["s"], [None]), Allreduce("a", 0, "c", 0, 5, "int32", "sum"),
            Allreduce("a", 0, "c", 0, 0, "int32", "sum")]]
    out.append(single_stream(1, b, ops, name="one-rank"))
    b = [{"x": as_bytes(np.array([r + 1, -(r + 2), 7 * r], np.int32)), "y": np.zeros(12, np.uint8)}
         for r in range(2)]
    ops = [[GroupStart(), GroupEnd(), Allreduce("x", 0, "y", 0, 0, "int32", "sum"),
            Allreduce("x", 0, "y", 0, 3, "int32", "max"), GroupStart(), GroupInit("e"),
            Start("e"), Start("e")] for _ in range(2)]
    out.append(single_stream(2, b, ops, name="empty-groups"))
    return out


def large_tag_program(grouped=False):
    """Tags that share low bits with rank numbers shifted into a packed key:
    (0 -> 1, tag 0) next to (0 -> 0, tag 2^24), (1 -> 0, tag 2^24 + 5) and
    the largest tag, 2^31 - 1.  Each channel must stay separate.  grouped:
    each rank's calls form one group."""
    big = 1 << 24
    b = [{"s": as_bytes(np.array([11, 22, 33], np.int32)), "r": np.zeros(12, np.uint8)},
         {"s": as_bytes(np.array([44, 55], np.int32)), "r": np.zeros(8, np.uint8)}]
    ops = [[Send("s", 0, 1, "int32", 1, 0, req="x"), Send("s", 4, 1, "int32", 0, big, req="y"),
            Recv("r", 0, 1, "int32", 0, big, status="self"),
            Recv("r", 4, 1, "int32", 1, big + 5, status="b5"),
            Recv("r", 8, 1, "int32", 1, (1 << 31) - 1, status="max"),
            Send("s", 8, 1, "int32", 1, (1 << 31) - 1),
            Wait(["x", "y"], [None, None])],
           [Recv("r", 0, 1, "int32", 0, 0, status="t0"),
            Send("s", 0, 1, "int32", 0, big + 5, req="z"),
            Send("s", 4, 1, "int32", 0, (1 << 31) - 1, req="w"),
            Recv("r", 4, 1, "int32", 0, (1 << 31) - 1, status="max"),
            Wait(["z", "w"], [None, None])]]
    if grouped:
        ops = [[GroupStart()] + o + [GroupEnd()] for o in ops]
    return single_stream(2, b, ops, name="large-tags" + ("-grouped" if grouped else ""))


# ------------------------------------------------------ grouped allreduces
def grouped_allreduces(nranks: int = 5, steps: int = 2, persistent: bool = False,
                       mismatch: bool = False) -> Program:
    """Each step one group holding messages around a ring and four
    allreduces (int32 SUM, float64 MIN, float32 SUM in place, a zero-count
    int64 MAX), each on buffers of its own; between steps every rank adds
    one to its int32 input, so each step reduces new values.  persistent:
    the group is recorded once (GroupInit) and started every step.
    mismatch: rank 1 groups its second allreduce with a different count,
    which fails the instance on every rank."""
    bufs, ops = [], []
    for r in range(nranks):
        g = rng(12, r)
        b = {"i32": as_bytes(g.integers(-2**30, 2**30, size=37, dtype=np.int64).astype(np.int32)),
             "o32": np.zeros(4 * 37, np.uint8),
             "f64": as_bytes(g.standard_normal(19)),
             "o64": np.zeros(8 * 19, np.uint8),
             "f32": as_bytes(g.standard_normal(101).astype(np.float32)),
             "s": as_bytes(np.arange(5, dtype=np.int32) + 100 * r),
             "h": np.zeros(20, np.uint8)}
        bufs.append(b)
        right, left = (r + 1) % nranks, (r - 1) % nranks
        n64 = 18 if (mismatch and r == 1) else 19
        body = [Send("s", 0, 5, "int32", right, 3, req="a"),
                Recv("h", 0, 5, "int32", left, 3, req="b"),
                Allreduce("i32", 0, "o32", 0, 37, "int32", "sum"),
                Allreduce("f64", 0, "o64", 0, n64, "float64", "min"),
                Allreduce(IN_PLACE, 0, "f32", 0, 101, "float32", "sum"),
                Allreduce("i32", 0, "o32", 0, 0, "int64", "max"),
                Wait(["a", "b"], [None, "st"])]
        bump = User(("add_const_i32", "i32", 0, 37, 1))
        lst = []
        if persistent:
            lst += [GroupStart()] + body + [GroupInit("g")]
            for _ in range(steps):
                lst += [Start("g"), bump]
        else:
            for _ in range(steps):
                lst += [GroupStart()] + body + [GroupEnd(), bump]
        ops.append(lst)
    name = "grouped-allreduce" + ("-persistent" if persistent else "") + ("-mismatch" if mismatch else "")
    return single_stream(nranks, bufs, ops, name=name)


def merged_allreduces(nranks: int = 6, steps: int = 2, persistent: bool = False,
                      chained: bool = False, messages: bool = True, big: int = 0) -> Program:
    """Each step one group whose allreduces are all float32 sums on buffers
    of their own: 3 elements (less than one 16-byte vector), 2501 elements
    (several 256-vector chunks and a one-element tail), 37 elements at a
    4-byte offset (not 16-byte aligned, so element by element), 700
    elements, 101 elements in place and a zero-count call; a message pair
    rides in the same group.  Between steps every rank adds one to the bit
    patterns of its inputs (a one-ulp change), so each step reduces new
    values.  chained: one more allreduce reads the 2501-element result, so
    two calls share bytes and must run in order.  persistent: the group is
    recorded once (GroupInit) and started every step.  messages=False: the
    group holds the allreduces only.  big: one more allreduce of that many
    elements (large groups take nontemporal accesses)."""
    specs = [("a", 3, 0), ("b", 2501, 0), ("c", 37, 4), ("d", 700, 0)]
    if big:
        specs.append(("g", big, 0))
    bufs, ops = [], []
    for r in range(nranks):
        g = rng(13, r)
        b = {}
        for name, cnt, off in specs:
            b[name + "i"] = np.concatenate(
                [np.zeros(off, np.uint8), as_bytes(g.standard_normal(cnt).astype(np.float32))])
            b[name + "o"] = np.zeros(off + 4 * cnt, np.uint8)
        b["ip"] = as_bytes(g.standard_normal(101).astype(np.float32))
        b["z"] = np.zeros(16, np.uint8)
        b["s"] = as_bytes(np.arange(3, dtype=np.int32) + 10 * r)
        b["h"] = np.zeros(12, np.uint8)
        if chained:
            b["eo"] = np.zeros(4 * 2501, np.uint8)
        bufs.append(b)
        right, left = (r + 1) % nranks, (r - 1) % nranks
        body = [Send("s", 0, 3, "int32", right, 7, req="a"),
                Recv("h", 0, 3, "int32", left, 7, req="b")] if messages else []
        body += [Allreduce(name + "i", off, name + "o", off, cnt, "float32", "sum")
                 for name, cnt, off in specs]
        body += [Allreduce(IN_PLACE, 0, "ip", 0, 101, "float32", "sum"),
                 Allreduce("ai", 0, "z", 0, 0, "float32", "sum")]
        if chained:
            body.append(Allreduce("bo", 0, "eo", 0, 2501, "float32", "sum"))
        if messages:
            body.append(Wait(["a", "b"], [None, "st"]))
        bump = [User(("add_const_i32", name + "i", off, cnt, 1)) for name, cnt, off in specs]
        lst = []
        if persistent:
            lst += [GroupStart()] + body + [GroupInit("g")]
            for _ in range(steps):
                lst += [Start("g")] + bump
        else:
            for _ in range(steps):
                lst += [GroupStart()] + body + [GroupEnd()] + bump
        ops.append(lst)
    name = ("merged-allreduce" + ("-persistent" if persistent else "") + ("-chained" if chained else "")
            + ("" if messages else "-no-messages") + (f"-big{big}" if big else ""))
    return single_stream(nranks, bufs, ops, name=name)
