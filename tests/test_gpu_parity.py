"""GPU parity: programs run through the libmpixs C ABI on the GPU must give
exactly the oracle's buffers, statuses and synchronous error codes.

Integer payloads, matching and ordering are compared bit for bit; float32
reductions are compared bit for bit as well, because both sides fold in
the canonical rank order with one IEEE rounding per step.
"""
import sys

import numpy as np
import pytest

from oracle import simulate as sim
from tests.gpu_runner import compare, run_program
from workloads import configs as C
from workloads.program import (
    ANY_SOURCE, ANY_TAG, Allreduce, Program, Recv, Send, Wait, as_bytes, single_stream,
)

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def check(p, cfg=None, host_synced=False, name=None):
    _say(name or p.name)
    ref = sim.run(p)
    assert not ref.deadlock, "test program must be safe"
    g = run_program(p, cfg=cfg, host_synced=host_synced)
    diffs = compare(p, g, ref)
    assert not diffs, "\n".join(diffs[:20])
    return g, ref


def check_stats(p, cfg=None, name=None):
    """check() that also reads the world's statistics before it is freed."""
    _say(name or p.name)
    ref = sim.run(p)
    assert not ref.deadlock, "test program must be safe"
    g = run_program(p, cfg=cfg, stats=True)
    diffs = compare(p, g, ref)
    assert not diffs, "\n".join(diffs[:20])
    return g, ref


def cfg_with(**kw):
    from paper_2208_13707_amd import mpixs as M
    c = M.Config()
    for k, v in kw.items():
        setattr(c, k, v)
    return c


# ------------------------------------------------------------------ config 1
def test_pingpong_small():
    check(C.pingpong(nmsg=20))


def test_pingpong_increment_full_size():
    g, _ = check(C.pingpong(nmsg=1000, increment=True))


# ------------------------------------------------------------- paper examples
def test_saxpy_example():
    g, _ = check(C.saxpy_example(n=4099))
    y = np.frombuffer(g.buffers[1]["y"].tobytes(), np.float32)
    assert np.all(y == 4.0)


def test_threads_example_four_streams_per_rank():
    check(C.threads_example(nthreads=4))


# ------------------------------------------------------------------ config 2
@pytest.mark.parametrize("count,steps,update,blocking", [
    (37, 4, False, True), (37, 4, True, False), (2730, 3, True, True), (5461, 2, False, False),
])
def test_ring_halo(count, steps, update, blocking):
    check(C.ring_halo(count=count, steps=steps, update=update, blocking_recv=blocking))


def test_ring_halo_full_size_message():
    """Largest configuration message (count 43690, 524,280 payload bytes)."""
    check(C.ring_halo(count=43690, steps=3, update=True))


@pytest.mark.parametrize("fuse", [-1, 1 << 30])
def test_ring_halo_fused_and_split_waits(fuse):
    check(C.ring_halo(count=2730, steps=3, update=True), cfg=cfg_with(fuse_max_bytes=fuse),
          name=f"halo fuse={fuse}")


# ------------------------------------------------------------------ config 3
@pytest.mark.parametrize("dtype", ["int64", "float32"])
@pytest.mark.parametrize("nbytes", [4096, 1 << 20])
def test_allreduce_sum(dtype, nbytes):
    check(C.allreduce(nbytes, dtype, nranks=16, calls=2))


@pytest.mark.parametrize("dtype", ["int64", "float32"])
def test_allreduce_sum_64mib(dtype):
    check(C.allreduce(64 << 20, dtype, nranks=16, calls=1))


@pytest.mark.parametrize("op", ["prod", "min", "max"])
@pytest.mark.parametrize("dtype", ["int32", "float64"])
def test_allreduce_other_ops(op, dtype):
    check(C.allreduce(12345 * 8, dtype, nranks=5, calls=1, op=op))


@pytest.mark.parametrize("nranks,dtype,op", [(8, "float32", "sum"), (32, "int64", "max"),
                                             (64, "int32", "sum"), (16, "float64", "prod")])
def test_allreduce_fixed_rank_count_kernels(nranks, dtype, op):
    """Split-path reductions over 8/16/32/64 ranks use the kernels unrolled
    over the rank count; odd element counts exercise the vector tail."""
    es = {"int32": 4, "int64": 8, "float32": 4, "float64": 8}[dtype]
    count = (4 << 20) // (es * nranks) * 2 + 3
    check(C.allreduce(count * es, dtype, nranks=nranks, calls=2, op=op))


def test_allreduce_in_place_and_ragged():
    check(C.allreduce(4 * 1001, "float32", nranks=7, calls=3, in_place=True))
    check(C.allreduce(8 * 3, "int64", nranks=3, calls=1))


# --------------------------------------------------------------- generality
@pytest.mark.parametrize("seed", range(8))
def test_random_programs(seed):
    check(C.random_program(seed, nranks=4, nmsg=40))


def test_random_program_many_ranks():
    check(C.random_program(100, nranks=12, nmsg=150, tags=5, ncomms=3, allreduces=3))


def test_batch_small():
    check(C.batch(npairs=300, nranks=8, max_bytes=65536))


# -------------------------------------------------------------- error paths
def test_truncation_type_mismatch_zero_count():
    b0 = {"s": as_bytes(np.arange(1, 11, dtype=np.int32))}
    b1 = {"r": np.full(64, 0xEE, np.uint8)}
    r0 = [Send("s", 0, 10, "int32", 1, 0), Send("s", 0, 3, "int32", 1, 1),
          Send("s", 0, 0, "int32", 1, 2)]
    r1 = [Recv("r", 0, 6, "int32", 0, 0, status="t"),
          Recv("r", 32, 3, "float32", 0, 1, status="m"),
          Recv("r", 48, 4, "int32", 0, 2, status="z")]
    g, _ = check(single_stream(2, [b0, b1], [r0, r1], name="errors"))
    assert g.stream_errors[1][0] == "ERR_TRUNCATE"
    assert g.stream_errors[0][0] == "SUCCESS"


def test_sync_errors_have_no_side_effects():
    b0 = {"s": as_bytes(np.array([9, 10], np.int32))}
    b1 = {"r": np.zeros(8, np.uint8)}
    r0 = [Send("s", 0, 1, "int32", 5, 0), Send("s", 0, 1, "int32", 1, -3),
          Send("s", 0, -1, "int32", 1, 0), Send("s", 0, 1, "complex", 1, 0),
          Send("s", 0, 1, "int32", 1, 0, comm=1),
          Send("s", 4, 1, "int32", 1, 0)]
    r1 = [Recv("r", 0, 1, "int32", ANY_SOURCE, 0), Recv("r", 0, 1, "int32", 0, ANY_TAG),
          Recv("r", 0, 1, ("vector", 2, 2, 1, "int32"), 0, 0),
          Recv("r", 4, 1, "int32", 0, 0, status="ok"), Wait(["nope"], [None])]
    check(Program(2, [b0, b1], [[r0], [r1]], 1, [[0, 0], [None, 0]], name="sync-errors"))


def test_waitall_across_streams_is_rejected():
    b0 = {"s": as_bytes(np.array([1, 2], np.int32))}
    b1 = {"r": np.zeros(8, np.uint8)}
    r0 = [[Send("s", 0, 1, "int32", 1, 0, comm=0, req="a"),
           Send("s", 4, 1, "int32", 1, 0, comm=1, req="b"),
           Wait(["a", "b"], [None, None]), Wait(["a"], [None]), Wait(["b"], [None])]]
    r1 = [[Recv("r", 0, 1, "int32", 0, 0, comm=0), Recv("r", 4, 1, "int32", 0, 0, comm=1)]]
    check(Program(2, [b0, b1], [r0, r1], 2, [[0, 0], [1, 1]], name="waitall-streams"))


def test_self_messages_and_tag_reordering():
    b = [{"s": as_bytes(np.arange(100, 106, dtype=np.int32)), "r": np.zeros(24, np.uint8)}]
    ops = [[Send("s", 0, 1, "int32", 0, 0, req="a"), Send("s", 4, 1, "int32", 0, 1, req="b"),
            Send("s", 8, 1, "int32", 0, 0, req="c"),
            Recv("r", 0, 1, "int32", 0, 1, status="x"), Recv("r", 4, 1, "int32", 0, 0),
            Recv("r", 8, 1, "int32", 0, 0), Wait(["a", "b", "c"], [None] * 3)]]
    g, _ = check(single_stream(1, b, ops, name="self"))
    assert np.frombuffer(g.buffers[0]["r"][:12].tobytes(), np.int32).tolist() == [101, 100, 102]


# ------------------------------------------------------ host-synced comparator
def test_host_synced_pingpong_matches():
    check(C.pingpong(nmsg=40, increment=True), host_synced=True, name="host-synced pingpong")


def test_host_synced_allreduce_matches():
    check(C.allreduce(1 << 16, "float32", nranks=16, calls=2), host_synced=True,
          name="host-synced allreduce")


def test_host_synced_vector_messages_match():
    count = 2730
    vt = C.halo_type(count)
    g = np.random.default_rng(5)
    bufs = [{"A": as_bytes(g.standard_normal(count * 8).astype(np.float32))},
            {"H": np.zeros(count * 32, np.uint8)}]
    ops = [[Send("A", 0, 1, vt, 1, 0), Send("A", 12, 1, vt, 1, 1)],
           [Recv("H", 0, 1, vt, 0, 0, status="a"), Recv("H", 12, 1, vt, 0, 1, status="b")]]
    check(single_stream(2, bufs, ops, name="host-synced vector"), host_synced=True)


# ----------------------------------------------------------------- batching
from workloads.program import GroupEnd, GroupStart  # noqa: E402


@pytest.mark.parametrize("count,blocking", [(37, True), (2730, False), (43690, True)])
def test_grouped_ring_halo(count, blocking):
    check(C.ring_halo(count=count, steps=3, update=True, blocking_recv=blocking, grouped=True))


@pytest.mark.parametrize("seed", range(4))
def test_grouped_random_programs(seed):
    check(C.random_program(seed, nranks=5, nmsg=60, grouped=True))


def test_grouped_batch_small():
    check(C.batch(npairs=400, nranks=8, max_bytes=65536, grouped=True))


def test_grouped_batch_config_size():
    """10,000 messages over 32 ranks in one group, as the batching workload."""
    check(C.batch(npairs=10000, nranks=32, grouped=True))


@pytest.mark.parametrize("npairs,nranks,runs", [(2048, 2, 0), (2305, 3, 0), (2305, 2, 2)])
def test_grouped_batch_planned_with_help(npairs, nranks, runs):
    """Groups from 2,048 pairs are planned in chunks of 256 pairs that the
    ranks waiting for the launch help with: the threshold itself with one
    helper, a ragged last chunk, and a persistent batch."""
    check(C.batch(npairs=npairs, nranks=nranks, max_bytes=4096, grouped=runs == 0, runs=runs),
          name=f"batch {npairs} pairs over {nranks} ranks ({'persistent' if runs else 'one group'})")


def test_group_head_to_head_and_unmatched():
    b = [{"s": as_bytes(np.array([10 + q, 20 + q], np.int32)), "r": np.full(8, 0xEE, np.uint8)}
         for q in range(2)]
    ops = [[GroupStart(), Send("s", 0, 1, "int32", 1 - q, 0),
            Recv("r", 0, 1, "int32", 1 - q, 0, status="st"), GroupEnd(),
            GroupStart(), Send("s", 4, 1, "int32", 1 - q, 5)] + ([GroupEnd()] if q else
                                                                   [Send("s", 4, 1, "int32", 1, 6),
                                                                    GroupEnd()])
           for q in range(2)]
    # rank 1 never receives tags 5/6 in its second group: that instance fails
    ops[1].insert(-1, Recv("r", 4, 1, "int32", 0, 5))
    g, _ = check(single_stream(2, b, ops, name="groups-h2h-unmatched"))
    assert np.frombuffer(g.buffers[1]["r"][:4].tobytes(), np.int32)[0] == 10


# ------------------------------------------------------- persistent batches
from workloads.program import GroupInit, Start  # noqa: E402


@pytest.mark.parametrize("count,blocking,graph,sync", [(37, True, 0, 0), (2730, False, 1, 0),
                                                       (43690, True, 0, 0), (37, False, 0, 1),
                                                       (43690, True, 0, 1)])
def test_persistent_ring_halo(count, blocking, graph, sync):
    check(C.ring_halo(count=count, steps=4, update=True, blocking_recv=blocking, persistent=True),
          cfg=cfg_with(batch_graph=graph, batch_sync=sync),
          name=f"persistent halo c{count} graph={graph} sync={sync}")


@pytest.mark.parametrize("tile,max_wg,graph,sync", [(1024, 4096, 0, 0), (256, 7, 1, 0),
                                                    (4096, 3, 0, 1), (512, 1 << 16, 1, 0),
                                                    (2048, 100, 0, 1)])
def test_persistent_batch_schedules(tile, max_wg, graph, sync):
    check(C.batch(npairs=400, nranks=8, max_bytes=65536, runs=3),
          cfg=cfg_with(batch_tile=tile, batch_max_wg=max_wg, batch_graph=graph, batch_sync=sync),
          name=f"persistent batch tile={tile} max_wg={max_wg} graph={graph} sync={sync}")


@pytest.mark.parametrize("graph,sync", [(1, 0), (0, 1)])
def test_persistent_batch_config_size(graph, sync):
    """10,000 messages over 32 ranks, planned once, started 3 times."""
    check(C.batch(npairs=10000, nranks=32, runs=3), cfg=cfg_with(batch_graph=graph, batch_sync=sync),
          name=f"persistent batch 10000 msgs graph={graph} sync={sync}")


def test_persistent_errors():
    b = [{"s": as_bytes(np.array([5, 6], np.int32)), "r": np.full(8, 0xEE, np.uint8)}
         for _ in range(2)]
    ops = [[GroupStart(), Send("s", 0, 1, "int32", 1, 0), Send("s", 4, 1, "int32", 1, 0),
            GroupInit("x"), Start("x")],
           [GroupStart(), Recv("r", 0, 1, "int32", 0, 0), GroupInit("x"), Start("x")]]
    check(single_stream(2, b, ops, name="persistent unmatched"))
    # the request left unwaited is released by a wait after the failed init
    ops = [[GroupStart(), Send("s", 0, 1, "int32", 1, 0, req="a"), GroupInit("y"), Start("y"),
            Wait(["a"], [None])],
           [GroupStart(), Recv("r", 0, 1, "int32", 0, 0), GroupInit("y"), Start("y")]]
    check(single_stream(2, b, ops, name="persistent unwaited"))


# -------------------------------------------------- ordered-queue matching
from tests.checks import check_competing  # noqa: E402


def queue_mode(p):
    p.matching = "queue"
    return p


@pytest.mark.parametrize("k", range(3))
def test_wildcard_programs(k):
    """Wildcard receives whose match is the same in every interleaving."""
    check(C.wildcard_programs()[k])


def test_wildcard_competing_senders():
    """Three senders race for ANY_SOURCE / ANY_TAG receives: every message
    arrives exactly once, in order per sender, with a matching status."""
    p = C.competing_senders()
    _say(p.name)
    for _ in range(3):
        g = run_program(p)
        vals = np.frombuffer(g.buffers[0]["r"].tobytes(), np.int32).tolist()
        check_competing(vals, [g.statuses[0][f"s{j}"] for j in range(12)])


@pytest.mark.parametrize("seed", range(4))
def test_queue_matching_random_programs(seed):
    """Without wildcards the queue engine must give sequence pairing's results."""
    check(queue_mode(C.random_program(seed, nranks=4, nmsg=40)), name=f"queue random {seed}")


def test_queue_matching_halo_and_batch():
    check(queue_mode(C.ring_halo(count=2730, steps=3, update=True, blocking_recv=False)),
          name="queue halo")
    check(queue_mode(C.batch(npairs=1000, nranks=8, max_bytes=65536)), name="queue batch")


# ------------------------------------------------------------ multiplex (§3.5)
from tests.checks import check_n_to_1_racing  # noqa: E402
from workloads.program import ANY_INDEX, GroupStart as _GroupStart  # noqa: E402


@pytest.mark.parametrize("nthreads", [2, 4, 8])
def test_multiplex_n_to_1_by_tag(nthreads):
    g, _ = check(C.multiplex_n_to_1(nthreads=nthreads, per=3))
    for k in range(3 * nthreads):
        v = int(np.frombuffer(g.buffers[1]["r"][4 * k: 4 * k + 4].tobytes(), np.int32)[0])
        assert g.status_index[1][f"s{k}"] == v // 100


def test_multiplex_n_to_1_racing():
    p = C.multiplex_n_to_1(nthreads=4, per=3, racing=True)
    _say(p.name)
    for _ in range(3):
        g = run_program(p)
        assert not any(g.sync_errors)
        vals = np.frombuffer(g.buffers[1]["r"].tobytes(), np.int32).tolist()
        check_n_to_1_racing(vals, [g.statuses[1][f"s{k}"] for k in range(12)],
                            indices=[g.status_index[1][f"s{k}"] for k in range(12)])


@pytest.mark.parametrize("n", [2, 3])
def test_multiplex_all_pairs(n):
    check(C.multiplex_all_pairs(n))


def test_multiplex_argument_errors():
    b = [{"s": as_bytes(np.array([1, 2], np.int32)), "r": np.zeros(8, np.uint8)} for _ in range(2)]
    ops = [[[Send("s", 0, 1, "int32", 1, 0),
             Send("s", 0, 1, "int32", 1, 0, src_idx=2, dst_idx=0),
             Send("s", 0, 1, "int32", 1, 0, src_idx=0, dst_idx=1),
             Allreduce("s", 0, "r", 0, 1, "int32", "sum"),
             _GroupStart(),
             Send("s", 4, 1, "int32", 1, 3, src_idx=1, dst_idx=0)]],
           [[Recv("r", 0, 1, "int32", 0, ANY_TAG, src_idx=ANY_INDEX, dst_idx=0, status="x")]]]
    check(Program(2, b, ops, 2, [[[0, 1], [0]]], name="multiplex-errors"))


# -------------------------------------------------------------- degenerate
@pytest.mark.parametrize("k", range(2))
def test_degenerate_programs(k):
    """A one-rank world (self messages, one-rank and zero-count allreduce);
    empty one-shot and persistent groups, zero-count allreduce."""
    check(C.degenerate_programs()[k])


@pytest.mark.parametrize("grouped", [False, True])
def test_large_tags_keep_channels_apart(grouped):
    """Channels whose tags share bits with shifted rank numbers stay apart."""
    check(C.large_tag_program(grouped))


# ------------------------------------------------------- grouped allreduces
@pytest.mark.parametrize("persistent,graph,sync", [(False, 0, 0), (True, 0, 0), (True, 1, 0),
                                                   (True, 0, 1)])
def test_grouped_allreduces(persistent, graph, sync):
    """Allreduces inside one-shot and persistent groups, with messages in the
    same groups; persistent runs launched one by one, as a graph, or ordered
    by events."""
    check(C.grouped_allreduces(persistent=persistent, steps=3),
          cfg=cfg_with(batch_graph=graph, batch_sync=sync),
          name=f"grouped allreduces persistent={persistent} graph={graph} sync={sync}")


@pytest.mark.parametrize("persistent", [False, True])
def test_grouped_allreduce_mismatch(persistent):
    check(C.grouped_allreduces(persistent=persistent, steps=1, mismatch=True))


@pytest.mark.parametrize("persistent,graph,sync,chained", [
    (False, 0, 0, False), (True, 0, 0, False), (True, 1, 0, False), (True, 0, 1, False),
    (False, 0, 0, True), (True, 1, 0, True),
])
def test_merged_allreduces(persistent, graph, sync, chained):
    """A group whose allreduces are all float32 sums on buffers of their own
    runs them as one merged reduce kernel (vector chunks, ragged tails, an
    unaligned buffer, fewer elements than a vector, in place, zero count);
    with a call that reads another's result they must run one by one."""
    steps = 3
    g, _ = check_stats(C.merged_allreduces(persistent=persistent, chained=chained, steps=steps),
                       cfg=cfg_with(batch_graph=graph, batch_sync=sync),
                       name=f"merged allreduces persistent={persistent} graph={graph} "
                            f"sync={sync} chained={chained}")
    # five nonzero allreduces per run of the group
    assert g.stats.reductions_merged == (0 if chained else 5 * steps)


@pytest.mark.parametrize("persistent,graph", [(False, 0), (True, 0), (True, 1)])
def test_merged_allreduces_without_messages(persistent, graph):
    """Groups of allreduces only: a persistent run launches no batch kernel."""
    g, _ = check_stats(C.merged_allreduces(persistent=persistent, steps=3, messages=False),
                       cfg=cfg_with(batch_graph=graph),
                       name=f"merged allreduces without messages persistent={persistent} graph={graph}")
    assert g.stats.reductions_merged == 5 * 3


def test_merged_allreduces_sixteen_ranks():
    g, _ = check_stats(C.merged_allreduces(nranks=16, steps=2), name="merged allreduces 16 ranks")
    assert g.stats.reductions_merged == 5 * 2


@pytest.mark.parametrize("persistent", [False, True])
def test_merged_allreduces_large(persistent):
    """16 ranks with one more allreduce of 600,001 float32 elements: the
    merged launch moves about 80 MB and takes nontemporal accesses."""
    g, _ = check_stats(C.merged_allreduces(nranks=16, steps=2, persistent=persistent, big=600_001),
                       name=f"merged allreduces large persistent={persistent}")
    assert g.stats.reductions_merged == 6 * 2
    assert g.stats.bytes_reduced >= 2 * (64 << 20)


def test_grouped_allreduces_fixed_rank_count():
    """16 ranks: the grouped reductions take the unrolled 16-rank kernel."""
    check(C.grouped_allreduces(nranks=16, steps=2))
