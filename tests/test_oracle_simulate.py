"""Pins of the oracle's program simulator (CPU only).

Expected values come from closed forms (an echo returns the data; +1 per
round trip adds the round-trip count), the paper's SAXPY example constants
(tests/golden/saxpy_example.txt), direct numpy slicing of the halo
exchange, payloads that encode their own send order, and programs whose
deadlock or completion is known by construction.
"""
import os

import numpy as np
import pytest

from oracle import simulate as sim
from workloads import configs as C
from workloads.program import (
    ANY_SOURCE, ANY_TAG, IN_PLACE, Allreduce, Program, Recv, Send, Wait, as_bytes,
    single_stream,
)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def i32(b):
    return np.frombuffer(b.tobytes(), np.int32)


def f32(b):
    return np.frombuffer(b.tobytes(), np.float32)


def test_pingpong_echo_returns_data():
    p = C.pingpong(nmsg=20)
    r = sim.run(p)
    assert not r.deadlock
    assert np.array_equal(r.buffers[0]["x"], p.buffers[0]["x"])
    assert len(r.match_log) == 20


def test_pingpong_increment_closed_form():
    p = C.pingpong(nmsg=1000, increment=True)
    r = sim.run(p)
    x0 = i32(p.buffers[0]["x"]).astype(np.int64)
    want = ((x0 + 500 + 2**31) % 2**32 - 2**31).astype(np.int32)
    assert np.array_equal(i32(r.buffers[0]["x"]), want)


def test_saxpy_example_value():
    vals = dict(line.split() for line in open(os.path.join(GOLDEN, "saxpy_example.txt"))
                if line.strip() and not line.startswith("#"))
    p = C.saxpy_example(n=1000)
    r = sim.run(p)
    y = f32(r.buffers[1]["y"])
    assert np.all(y == np.float32(vals["result"]))
    assert np.all(f32(r.buffers[1]["x"]) == np.float32(vals["x"]))


def _halo_by_slicing(p, steps, count, update):
    """The ring halo exchange written with numpy slicing of [count, 8] rows."""
    n = p.nranks
    A = [f32(b["A"]).reshape(count, 8).copy() for b in p.buffers]
    H = [f32(b["H"]).reshape(count, 8).copy() for b in p.buffers]
    for _ in range(steps):
        newH = [h.copy() for h in H]
        for r in range(n):
            newH[r][:, 0:3] = A[(r - 1) % n][:, 0:3]
            newH[r][:, 3:6] = A[(r + 1) % n][:, 3:6]
        H = newH
        if update:
            for r in range(n):
                A[r][:, 0:6] += H[r][:, 0:6]
    return A, H


@pytest.mark.parametrize("update,blocking", [(False, True), (True, True), (True, False)])
def test_ring_halo_matches_slicing(update, blocking):
    count, steps = 37, 4
    p = C.ring_halo(count=count, steps=steps, update=update, blocking_recv=blocking)
    r = sim.run(p)
    assert not r.deadlock
    A, H = _halo_by_slicing(p, steps, count, update)
    for q in range(p.nranks):
        assert np.array_equal(f32(r.buffers[q]["A"]).reshape(count, 8), A[q])
        assert np.array_equal(f32(r.buffers[q]["H"]).reshape(count, 8), H[q])
        st = r.statuses[q][f"st{steps - 1}a"]
        assert st == ((q - 1) % p.nranks, steps - 1, "SUCCESS", 12 * count)


def _order_program(tags_send, tags_recv, blocking_send):
    """Rank 0 sends payload i (one int32) with tag tags_send[i]; rank 1
    receives with tags_recv, each into its own slot."""
    n = len(tags_send)
    b0 = {"s": as_bytes(np.arange(100, 100 + n, dtype=np.int32))}
    b1 = {"r": np.zeros(4 * n, np.uint8)}
    r0 = []
    for i, t in enumerate(tags_send):
        r0.append(Send("s", 4 * i, 1, "int32", 1, t, req=None if blocking_send else f"q{i}"))
    if not blocking_send:
        r0.append(Wait([f"q{i}" for i in range(n)], [None] * n))
    r1 = [Recv("r", 4 * i, 1, "int32", 0, t, status=f"st{i}") for i, t in enumerate(tags_recv)]
    return single_stream(2, [b0, b1], [r0, r1])


def test_non_overtaking_same_channel():
    p = _order_program([5] * 10, [5] * 10, blocking_send=True)
    r = sim.run(p)
    assert i32(r.buffers[1]["r"]).tolist() == list(range(100, 110))


def test_tags_match_independently():
    # sends a(tag0) b(tag1) c(tag0); receives tag1, tag0, tag0
    p = _order_program([0, 1, 0], [1, 0, 0], blocking_send=False)
    r = sim.run(p)
    assert not r.deadlock
    assert i32(r.buffers[1]["r"]).tolist() == [101, 100, 102]
    # the same with blocking (synchronous) sends cannot complete
    p = _order_program([0, 1, 0], [1, 0, 0], blocking_send=True)
    assert sim.run(p).deadlock


def test_communicators_match_independently():
    b0 = {"s": as_bytes(np.array([7, 8], np.int32))}
    b1 = {"r": np.zeros(8, np.uint8)}
    r0 = [Send("s", 0, 1, "int32", 1, 0, comm=0, req="a"),
          Send("s", 4, 1, "int32", 1, 0, comm=1, req="b"), Wait(["a", "b"], [None, None])]
    r1 = [Recv("r", 0, 1, "int32", 0, 0, comm=1), Recv("r", 4, 1, "int32", 0, 0, comm=0)]
    p = single_stream(2, [b0, b1], [r0, r1], ncomms=2)
    r = sim.run(p)
    assert i32(r.buffers[1]["r"]).tolist() == [8, 7]


def test_head_to_head_blocking_sends_deadlock():
    b = [{"s": np.zeros(4, np.uint8), "r": np.zeros(4, np.uint8)} for _ in range(2)]
    ops = [[Send("s", 0, 1, "int32", 1 - q, 0), Recv("r", 0, 1, "int32", 1 - q, 0)]
           for q in range(2)]
    r = sim.run(single_stream(2, b, ops))
    assert r.deadlock and len(r.blocked) == 2
    ops = [[Send("s", 0, 1, "int32", 1 - q, 0, req="x"), Recv("r", 0, 1, "int32", 1 - q, 0),
            Wait(["x"], [None])] for q in range(2)]
    assert not sim.run(single_stream(2, b, ops)).deadlock


def test_self_message_with_isend():
    b = [{"s": as_bytes(np.array([42], np.int32)), "r": np.zeros(4, np.uint8)}]
    ops = [[Send("s", 0, 1, "int32", 0, 3, req="x"), Recv("r", 0, 1, "int32", 0, 3),
            Wait(["x"], [None])]]
    r = sim.run(single_stream(1, b, ops))
    assert i32(r.buffers[0]["r"]).tolist() == [42]
    ops = [[Send("s", 0, 1, "int32", 0, 3), Recv("r", 0, 1, "int32", 0, 3)]]
    assert sim.run(single_stream(1, b, ops)).deadlock


def test_truncation_and_type_mismatch_and_zero_count():
    b0 = {"s": as_bytes(np.arange(1, 11, dtype=np.int32))}
    b1 = {"r": np.full(64, 0xEE, np.uint8)}
    r0 = [Send("s", 0, 10, "int32", 1, 0), Send("s", 0, 3, "int32", 1, 1),
          Send("s", 0, 0, "int32", 1, 2)]
    r1 = [Recv("r", 0, 6, "int32", 0, 0, status="t"),
          Recv("r", 32, 3, "float32", 0, 1, status="m"),
          Recv("r", 48, 4, "int32", 0, 2, status="z")]
    r = sim.run(single_stream(2, [b0, b1], [r0, r1]))
    assert r.statuses[1]["t"] == (0, 0, "ERR_TRUNCATE", 24)
    assert i32(r.buffers[1]["r"][:24]).tolist() == [1, 2, 3, 4, 5, 6]
    assert r.buffers[1]["r"][24:32].tolist() == [0xEE] * 8
    assert r.statuses[1]["m"] == (0, 1, "ERR_TYPE", 0)
    assert r.buffers[1]["r"][32:44].tolist() == [0xEE] * 12
    assert r.statuses[1]["z"] == (0, 2, "SUCCESS", 0)


def test_sync_errors_have_no_side_effects():
    b0 = {"s": as_bytes(np.array([9, 10], np.int32))}
    b1 = {"r": np.zeros(8, np.uint8)}
    r0 = [Send("s", 0, 1, "int32", 5, 0),          # bad rank
          Send("s", 0, 1, "int32", 1, -3),         # bad tag
          Send("s", 0, -1, "int32", 1, 0),         # bad count
          Send("s", 0, 1, "complex", 1, 0),        # bad type
          Send("s", 0, 1, "int32", 1, 0, comm=1),  # comm without a stream here
          Send("s", 4, 1, "int32", 1, 0)]
    r1 = [Recv("r", 0, 1, "int32", ANY_SOURCE, 0),
          Recv("r", 0, 1, "int32", 0, ANY_TAG),
          Recv("r", 0, 1, ("vector", 2, 2, 1, "int32"), 0, 0),   # overlapping receive
          Recv("r", 4, 1, "int32", 0, 0, status="ok"),
          Wait(["nope"], [None])]
    p = Program(2, [b0, b1], [[r0], [r1]], 1, [[0, 0], [None, 0]])
    r = sim.run(p)
    assert [e for _, _, e in r.sync_errors[0]] == [
        "ERR_RANK", "ERR_TAG", "ERR_COUNT", "ERR_TYPE", "ERR_COMM"]
    assert [e for _, _, e in r.sync_errors[1]] == [
        "ERR_RANK", "ERR_TAG", "ERR_TYPE", "ERR_REQUEST"]
    assert i32(r.buffers[1]["r"]).tolist() == [0, 10]
    assert r.statuses[1]["ok"] == (0, 0, "SUCCESS", 4)
    assert len(r.match_log) == 1 and r.match_log[0][-1] == 0


def test_waitall_across_streams_is_an_error():
    b0 = {"s": as_bytes(np.array([1, 2], np.int32))}
    b1 = {"r": np.zeros(8, np.uint8)}
    r0 = [[Send("s", 0, 1, "int32", 1, 0, comm=0, req="a"),
           Send("s", 4, 1, "int32", 1, 0, comm=1, req="b"),
           Wait(["a", "b"], [None, None]), Wait(["a"], [None]), Wait(["b"], [None])]]
    r1 = [[Recv("r", 0, 1, "int32", 0, 0, comm=0), Recv("r", 4, 1, "int32", 0, 0, comm=1)]]
    p = Program(2, [b0, b1], [r0, r1], 2, [[0, 0], [1, 1]])
    r = sim.run(p)
    assert [e for _, _, e in r.sync_errors[0]] == ["ERR_STREAM"]
    assert not r.deadlock


def test_threads_example_each_pair_delivers():
    p = C.threads_example(nthreads=4)
    r = sim.run(p)
    for i in range(4):
        assert np.array_equal(r.buffers[1][f"buf{i}"], p.buffers[0][f"buf{i}"])


@pytest.mark.parametrize("in_place", [False, True])
def test_allreduce_closed_form(in_place):
    n, count = 16, 100
    base = (np.arange(count, dtype=np.int64) - 50) * (2**33)
    bufs, ops = [], []
    for q in range(n):
        if in_place:
            bufs.append({"x": as_bytes(base + q)})
            ops.append([Allreduce(IN_PLACE, 0, "x", 0, count, "int64", "sum")])
        else:
            bufs.append({"s": as_bytes(base + q), "x": np.zeros(8 * count, np.uint8)})
            ops.append([Allreduce("s", 0, "x", 0, count, "int64", "sum")])
    r = sim.run(single_stream(n, bufs, ops))
    for q in range(n):
        assert np.array_equal(np.frombuffer(r.buffers[q]["x"].tobytes(), np.int64),
                              16 * base + 120)


def test_allreduce_instances_pair_in_order():
    # two allreduces per rank; rank q contributes q+1 then 10*(q+1)
    n = 4
    bufs, ops = [], []
    for q in range(n):
        bufs.append({"a": as_bytes(np.array([q + 1], np.int32)),
                     "b": as_bytes(np.array([10 * (q + 1)], np.int32)),
                     "x": np.zeros(4, np.uint8), "y": np.zeros(4, np.uint8)})
        ops.append([Allreduce("a", 0, "x", 0, 1, "int32", "sum"),
                    Allreduce("b", 0, "y", 0, 1, "int32", "sum")])
    r = sim.run(single_stream(n, bufs, ops))
    assert all(i32(r.buffers[q]["x"])[0] == 10 and i32(r.buffers[q]["y"])[0] == 100
               for q in range(n))


@pytest.mark.parametrize("seed", range(6))
def test_random_programs_complete_and_deliver(seed):
    p = C.random_program(seed)
    r = sim.run(p)
    assert not r.deadlock
    # each message's packed payload lands in its own receive region: check by
    # re-reading the send regions with numpy views of the vector/contiguous types
    assert len(r.match_log) == 40
    assert all(not e for e in r.sync_errors)


# ------------------------------------------------------------------- groups
from workloads.program import GroupEnd, GroupStart  # noqa: E402


def test_group_head_to_head_blocking_sends_complete():
    b = [{"s": as_bytes(np.array([10 + q], np.int32)), "r": np.zeros(4, np.uint8)}
         for q in range(2)]
    ops = [[GroupStart(), Send("s", 0, 1, "int32", 1 - q, 0), Recv("r", 0, 1, "int32", 1 - q, 0,
                                                                    status="st"),
            GroupEnd()] for q in range(2)]
    r = sim.run(single_stream(2, b, ops))
    assert not r.deadlock
    assert [i32(r.buffers[q]["r"])[0] for q in range(2)] == [11, 10]
    assert r.statuses[0]["st"] == (1, 0, "SUCCESS", 4)


def test_group_unmatched_fails_whole_instance():
    b = [{"s": as_bytes(np.array([1, 2], np.int32)), "r": np.full(8, 0xEE, np.uint8)}
         for _ in range(2)]
    ops = [[GroupStart(), Send("s", 0, 1, "int32", 1, 0), Send("s", 4, 1, "int32", 1, 1),
            GroupEnd()],
           [GroupStart(), Recv("r", 0, 1, "int32", 0, 0), GroupEnd()]]
    r = sim.run(single_stream(2, b, ops))
    assert not r.deadlock
    assert [e for _, _, e in r.sync_errors[0]] == ["ERR_ARG"]
    assert [e for _, _, e in r.sync_errors[1]] == ["ERR_ARG"]
    assert r.buffers[1]["r"].tolist() == [0xEE] * 8


@pytest.mark.parametrize("blocking", [True, False])
def test_grouped_halo_equals_slicing(blocking):
    count, steps = 29, 3
    p = C.ring_halo(count=count, steps=steps, update=True, blocking_recv=blocking, grouped=True)
    r = sim.run(p)
    assert not r.deadlock
    A, H = _halo_by_slicing(p, steps, count, True)
    for q in range(p.nranks):
        assert np.array_equal(f32(r.buffers[q]["A"]).reshape(count, 8), A[q])
        assert r.statuses[q][f"st{steps - 1}b"] == ((q + 1) % p.nranks, steps - 1, "SUCCESS",
                                                     12 * count)


@pytest.mark.parametrize("seed", range(3))
def test_grouped_random_program_equals_ungrouped(seed):
    a = sim.run(C.random_program(seed))
    b = sim.run(C.random_program(seed, grouped=True))
    assert not b.deadlock
    for q in range(len(a.buffers)):
        for k in a.buffers[q]:
            assert np.array_equal(a.buffers[q][k], b.buffers[q][k])
        assert a.statuses[q] == b.statuses[q]


# ------------------------------------------------------------ persistent groups
from workloads.program import GroupInit, Start, User  # noqa: E402


@pytest.mark.parametrize("blocking", [True, False])
def test_persistent_halo_equals_slicing(blocking):
    """A halo step recorded once and started every step gives the exchange
    written with numpy slicing."""
    count, steps = 31, 4
    p = C.ring_halo(count=count, steps=steps, update=True, blocking_recv=blocking,
                    persistent=True)
    r = sim.run(p)
    assert not r.deadlock and not any(r.sync_errors)
    A, H = _halo_by_slicing(p, steps, count, True)
    for q in range(p.nranks):
        assert np.array_equal(f32(r.buffers[q]["A"]).reshape(count, 8), A[q])
        assert np.array_equal(f32(r.buffers[q]["H"]).reshape(count, 8), H[q])
        assert r.statuses[q]["stb"] == ((q + 1) % p.nranks, 0, "SUCCESS", 12 * count)


def test_persistent_batch_moves_the_last_contents():
    """Each run re-reads the send buffers: after the last of 3 runs (the
    senders add 1 to every int32 word between runs) every contiguous
    message's receive bytes equal the sender's final bytes, computed with
    numpy alone."""
    runs = 3
    p = C.batch(npairs=150, nranks=5, max_bytes=2048, runs=runs)
    r = sim.run(p)
    assert not r.deadlock and not any(r.sync_errors)
    final = []
    for q in range(p.nranks):
        w = p.buffers[q]["sbuf"].view(np.int32).copy()
        w += np.int32(runs - 1)
        final.append(w.view(np.uint8))
    sends, recvs = {}, {}
    for q in range(p.nranks):
        for o in p.ops[q][0]:
            if isinstance(o, Send):
                sends[o.req[1:]] = (q, o)
            elif isinstance(o, Recv):
                recvs[o.req[1:]] = (q, o)
    checked = 0
    for i, (s, so) in sends.items():
        d, ro = recvs[i]
        if isinstance(so.dtype, str):
            n = so.count * {"uint8": 1, "int32": 4, "float32": 4}[so.dtype]
            got = r.buffers[d]["rbuf"][ro.off: ro.off + n]
            assert np.array_equal(got, final[s][so.off: so.off + n]), i
            checked += 1
    assert checked > 50


def test_persistent_unmatched_or_unwaited_init_fails():
    b = [{"s": as_bytes(np.array([5, 6], np.int32)), "r": np.full(8, 0xEE, np.uint8)}
         for _ in range(2)]
    # rank 0 records one send too many: init fails everywhere, starts are
    # invalid and nothing moves
    ops = [[GroupStart(), Send("s", 0, 1, "int32", 1, 0), Send("s", 4, 1, "int32", 1, 0),
            GroupInit("x"), Start("x")],
           [GroupStart(), Recv("r", 0, 1, "int32", 0, 0), GroupInit("x"), Start("x")]]
    r = sim.run(single_stream(2, b, ops))
    assert not r.deadlock
    assert r.sync_errors[0] == [(0, 3, "ERR_ARG"), (0, 4, "ERR_REQUEST")]
    assert r.sync_errors[1] == [(0, 2, "ERR_ARG"), (0, 3, "ERR_REQUEST")]
    assert r.buffers[1]["r"].tolist() == [0xEE] * 8
    # a request created in the group and never waited inside it
    ops = [[GroupStart(), Send("s", 0, 1, "int32", 1, 0, req="a"), GroupInit("y"), Start("y"),
            Wait(["a"], [None])],
           [GroupStart(), Recv("r", 0, 1, "int32", 0, 0), GroupInit("y"), Start("y")]]
    r = sim.run(single_stream(2, b, ops))
    assert r.sync_errors[0] == [(0, 2, "ERR_ARG"), (0, 3, "ERR_REQUEST")]
    assert r.sync_errors[1][0] == (0, 2, "ERR_ARG")
    assert r.buffers[1]["r"].tolist() == [0xEE] * 8


def test_persistent_runs_equal_repeated_groups():
    """Start == GroupStart + the recorded operations + GroupEnd, run by run
    (a planted mistake that snapshots payloads at init fails the batch test
    above; this one checks statuses and buffers against one-shot groups)."""
    p = C.batch(npairs=80, nranks=4, max_bytes=1024, runs=2)
    q = C.batch(npairs=80, nranks=4, max_bytes=1024, grouped=True)
    unrolled = []
    for rank in range(q.nranks):
        body = q.ops[rank][0]
        sb = q.buffers[rank]["sbuf"]
        unrolled.append(body + [User(("add_const_i32", "sbuf", 0, sb.size // 4, 1))] + body)
    u = single_stream(q.nranks, q.buffers, unrolled)
    a, b = sim.run(p), sim.run(u)
    for rank in range(p.nranks):
        for k in a.buffers[rank]:
            assert np.array_equal(a.buffers[rank][k], b.buffers[rank][k])
        assert a.statuses[rank] == b.statuses[rank]


# ------------------------------------------------------------------ wildcards
from tests.checks import check_competing  # noqa: E402


def i32(a):
    return np.frombuffer(a.tobytes(), np.int32)


def _queue(nranks, bufs, ops, name="wild"):
    p = single_stream(nranks, bufs, ops, name=name)
    p.matching = "queue"
    return p

def test_wildcard_matches_in_order():
    p1, p2, p3 = C.wildcard_programs()
    r = sim.run(p1)
    assert not r.deadlock and not any(r.sync_errors)
    assert i32(r.buffers[1]["r"]).tolist() == [50, 30, 70]
    assert [r.statuses[1][f"st{i}"][:2] for i in range(3)] == [(0, 5), (0, 3), (0, 7)]
    r = sim.run(p2)
    assert i32(r.buffers[1]["r"]).tolist() == [102, 100]
    assert r.statuses[1]["a"] == (2, 20, "SUCCESS", 4) and r.statuses[1]["b"] == (0, 10, "SUCCESS", 4)
    r = sim.run(p3)
    assert i32(r.buffers[1]["r"]).tolist() == [1, 2]
    assert r.statuses[1]["sw"] == (0, 4, "SUCCESS", 4)


def test_wildcard_competing_senders_are_valid():
    p = C.competing_senders()
    r = sim.run(p)
    assert not r.deadlock
    vals = i32(r.buffers[0]["r"]).tolist()
    check_competing(vals, [r.statuses[0][f"s{j}"] for j in range(12)])


def test_wildcards_rejected_in_sequence_mode_and_in_groups():
    b = [{"s": as_bytes(np.array([1], np.int32))}, {"r": np.zeros(4, np.uint8)}]
    ops = [[Send("s", 0, 1, "int32", 1, 0)],
           [Recv("r", 0, 1, "int32", ANY_SOURCE, 0), Recv("r", 0, 1, "int32", 0, 0)]]
    r = sim.run(single_stream(2, b, ops))
    assert r.sync_errors[1] == [(0, 0, "ERR_RANK")]
    ops = [[GroupStart(), GroupEnd(), Send("s", 0, 1, "int32", 1, 0)],
           [GroupStart(), Recv("r", 0, 1, "int32", 0, ANY_TAG), GroupEnd(),
            Recv("r", 0, 1, "int32", 0, 0)]]
    r = sim.run(_queue(2, b, ops))
    assert not r.deadlock
    assert r.sync_errors[1] == [(0, 1, "ERR_TAG")]
    assert i32(r.buffers[1]["r"]).tolist() == [1]


def test_queue_matching_without_wildcards_equals_sequence_pairing():
    """Without wildcards both matching modes are MPI's non-overtaking rule."""
    for seed in range(4):
        a = sim.run(C.random_program(seed))
        q = C.random_program(seed)
        q.matching = "queue"
        b = sim.run(q)
        for rank in range(len(a.buffers)):
            for k in a.buffers[rank]:
                assert np.array_equal(a.buffers[rank][k], b.buffers[rank][k])
            assert a.statuses[rank] == b.statuses[rank]


# ------------------------------------------------------------ multiplex (§3.5)
from tests.checks import check_n_to_1_racing  # noqa: E402
from workloads.program import ANY_INDEX  # noqa: E402


def test_multiplex_n_to_1_by_tag():
    p = C.multiplex_n_to_1(nthreads=4, per=3)
    r = sim.run(p)
    assert not r.deadlock and not any(r.sync_errors)
    want = [100 * i + j for i in range(4) for j in range(3)][::-1]
    assert i32(r.buffers[1]["r"]).tolist() == want
    assert r.statuses[1]["s0"] == (0, 32, "SUCCESS", 4)


def test_multiplex_n_to_1_racing_is_valid():
    p = C.multiplex_n_to_1(nthreads=4, per=3, racing=True)
    r = sim.run(p)
    assert not r.deadlock
    check_n_to_1_racing(i32(r.buffers[1]["r"]).tolist(), [r.statuses[1][f"s{k}"] for k in range(12)])


def test_multiplex_all_pairs_closed_form():
    n = 3
    r = sim.run(C.multiplex_all_pairs(n))
    assert not r.deadlock and not any(r.sync_errors)
    for rank in range(2):
        got = i32(r.buffers[rank]["r"]).tolist()
        # thread i received from thread j of the other rank: 1000 * (1 - rank) + 10 * j + i
        assert got == [1000 * (1 - rank) + 10 * j + i for i in range(n) for j in range(n)]


def test_multiplex_argument_errors():
    b = [{"s": as_bytes(np.array([1, 2], np.int32)), "r": np.zeros(8, np.uint8)} for _ in range(2)]
    ops = [[[Send("s", 0, 1, "int32", 1, 0),                                  # ordinary: ERR_COMM
             Send("s", 0, 1, "int32", 1, 0, src_idx=2, dst_idx=0),            # local index: ERR_RANK
             Send("s", 0, 1, "int32", 1, 0, src_idx=0, dst_idx=1),            # remote index: ERR_RANK
             Allreduce("s", 0, "r", 0, 1, "int32", "sum"),                    # ERR_COMM
             GroupStart(),                                                    # ERR_COMM
             Send("s", 4, 1, "int32", 1, 3, src_idx=1, dst_idx=0)]],
           [[Recv("r", 0, 1, "int32", 0, ANY_TAG, src_idx=ANY_INDEX, dst_idx=0, status="x")]]]
    p = Program(2, b, ops, 2, [[[0, 1], [0]]], name="mp-errors")
    r = sim.run(p)
    assert not r.deadlock
    assert r.sync_errors[0] == [(0, 0, "ERR_COMM"), (0, 1, "ERR_RANK"), (0, 2, "ERR_RANK"),
                                (0, 3, "ERR_COMM"), (0, 4, "ERR_COMM")]
    assert i32(r.buffers[1]["r"]).tolist()[0] == 2
    assert r.statuses[1]["x"] == (0, 3, "SUCCESS", 4)


def test_degenerate_programs():
    """One rank: a message to itself is delivered, an allreduce over one rank
    is the identity, a zero-count allreduce writes nothing; empty groups,
    one-shot and persistent, move nothing."""
    one, two = C.degenerate_programs()
    r = sim.run(one)
    assert not r.deadlock and not any(r.sync_errors)
    assert i32(r.buffers[0]["b"]).tolist() == [1, 2, 3, 4, 5]
    assert i32(r.buffers[0]["c"]).tolist() == [1, 2, 3, 4, 5]
    assert r.statuses[0]["st"] == (0, 7, "SUCCESS", 20)
    r = sim.run(two)
    assert not r.deadlock and not any(r.sync_errors)
    for q in range(2):
        assert i32(r.buffers[q]["y"]).tolist() == [2, -2, 7]
        assert i32(r.buffers[q]["x"]).tolist() == [q + 1, -(q + 2), 7 * q]


@pytest.mark.parametrize("grouped", [False, True])
def test_large_tags_keep_channels_apart(grouped):
    r = sim.run(C.large_tag_program(grouped))
    assert not r.deadlock and not any(r.sync_errors)
    assert i32(r.buffers[0]["r"]).tolist() == [22, 44, 55]
    assert i32(r.buffers[1]["r"]).tolist() == [11, 33]
    assert r.statuses[0]["self"] == (0, 1 << 24, "SUCCESS", 4)
    assert r.statuses[0]["b5"] == (1, (1 << 24) + 5, "SUCCESS", 4)
    assert r.statuses[1]["max"] == (0, (1 << 31) - 1, "SUCCESS", 4)


# ------------------------------------------------------- grouped allreduces
def _ungrouped(p):
    """The same program with every group marker removed and each persistent
    start replaced by the recorded calls."""
    out = []
    for r in range(p.nranks):
        ops = p.ops[r][0]
        rec, lst, recording = [], [], False
        for o in ops:
            if isinstance(o, GroupStart):
                recording, rec = True, []
            elif isinstance(o, GroupEnd):
                recording = False
                lst += rec
            elif isinstance(o, GroupInit):
                recording = False
            elif isinstance(o, Start):
                lst += rec
            elif recording:
                rec.append(o)
            else:
                lst.append(o)
        out.append([lst])
    q = Program(p.nranks, p.copy_buffers(), out, p.streams_per_rank, p.comm_streams, name="flat")
    return q


@pytest.mark.parametrize("persistent", [False, True])
def test_grouped_allreduces_equal_the_calls_in_order(persistent):
    """Grouped allreduces (one-shot and persistent) give the buffers of the
    same calls issued one by one, and the float32 in-place sum equals a
    sequential float32 fold written out here."""
    p = C.grouped_allreduces(persistent=persistent, steps=3)
    a, b = sim.run(p), sim.run(_ungrouped(p))
    assert not a.deadlock and not any(a.sync_errors) and not b.deadlock
    for q in range(p.nranks):
        for k in a.buffers[q]:
            assert np.array_equal(a.buffers[q][k], b.buffers[q][k]), (q, k)
    # three in-place sums of the ranks' float32 vectors, folded in rank order
    x = [p.buffers[q]["f32"].view(np.float32).copy() for q in range(p.nranks)]
    for _ in range(3):
        acc = x[0].copy()
        for q in range(1, p.nranks):
            acc = (acc + x[q]).astype(np.float32)
        x = [acc.copy() for _ in range(p.nranks)]
    assert np.array_equal(a.buffers[0]["f32"].view(np.float32), x[0])


@pytest.mark.parametrize("persistent,chained,messages", [
    (False, False, True), (True, False, True), (False, True, True), (True, True, True),
    (True, False, False)])
def test_merged_allreduces_equal_the_calls_in_order(persistent, chained, messages):
    """A group of float32 sums only (the kind the library may run as one
    kernel) gives the buffers of the same calls issued one by one; the
    2501-element result equals a float32 fold in rank order written out
    here, with the inputs bumped by one ulp pattern between steps, and the
    chained call (which reads that result) sees the final value of the same
    step."""
    steps = 2
    p = C.merged_allreduces(persistent=persistent, chained=chained, steps=steps, messages=messages)
    a, b = sim.run(p), sim.run(_ungrouped(p))
    assert not a.deadlock and not any(a.sync_errors) and not b.deadlock
    for q in range(p.nranks):
        for k in a.buffers[q]:
            assert np.array_equal(a.buffers[q][k], b.buffers[q][k]), (q, k)
    x = [p.buffers[q]["bi"].view(np.int32).copy() for q in range(p.nranks)]
    for step in range(steps):
        acc = x[0].view(np.float32).copy()
        for q in range(1, p.nranks):
            acc = (acc + x[q].view(np.float32)).astype(np.float32)
        x = [v + np.int32(1) for v in x]
    for q in range(p.nranks):
        assert np.array_equal(a.buffers[q]["bo"].view(np.float32), acc)
        assert not a.buffers[q]["z"].any()
        if chained:
            chain = acc.copy()
            for _ in range(1, p.nranks):
                chain = (chain + acc).astype(np.float32)
            assert np.array_equal(a.buffers[q]["eo"].view(np.float32), chain)


@pytest.mark.parametrize("persistent", [False, True])
def test_grouped_allreduce_mismatch_fails_the_instance(persistent):
    p = C.grouped_allreduces(persistent=persistent, steps=1, mismatch=True)
    r = sim.run(p)
    assert not r.deadlock
    errs = [[e for _, _, e in r.sync_errors[q]] for q in range(p.nranks)]
    if persistent:
        # GroupInit fails on every rank, and the start of the failed batch
        assert all(e == ["ERR_ARG", "ERR_REQUEST"] for e in errs)
    else:
        assert all(e == ["ERR_ARG"] for e in errs)
    for q in range(p.nranks):
        assert not r.buffers[q]["o32"].any() and not r.buffers[q]["h"].any()
