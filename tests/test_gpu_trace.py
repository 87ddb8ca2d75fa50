"""Device event trace (§3.4: enqueued operations run on the stream; the trace
records when each of their steps happened there), through the C ABI.

Every nonblocking message leaves four events in the world's ring, all on
its channel block and with the message's counter value:
POST (the first side's stream published its ready word), MATCH (the other
side's stream saw it, on that same word), DONE (the copying stream published
done) and COMPLETE (the first side's stream saw done).  Their times do not
decrease in that order, the copying stream records MATCH and DONE, and the
first side's stream POST and COMPLETE.  Checked on the fused (4 KiB) and
split (128 KiB) copy paths with 2 ranks, and on an allreduce: the non-last
rank's arrival is a POST matched by the reducing rank, whose DONE the other
rank completes.  A persistent batch leaves, for run e, every other rank's
arrival (POST, value e), the launching rank's wait seeing each (MATCH), one
DONE after the batch kernel and every other rank's COMPLETE, in that order,
and each rank's next arrival after its completion.  A ring smaller than the
events keeps the newest ones, and a world without tracing refuses the read.
"""
import sys
from collections import defaultdict

import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def _cfg(**kw):
    from paper_2208_13707_amd import mpixs as M
    c = M.Config()
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def _messages(D, M, sess, n, count, tag0):
    import torch
    src = torch.arange(n * count, dtype=torch.int32, device="cuda")
    dst = torch.zeros(n * count, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    r0 = [dict(kind=D.ISEND, peer=1, tag=tag0 + i, count=count, datatype=M.INT32,
               buf=src.data_ptr() + 4 * count * i, req=i) for i in range(n)]
    r0.append(dict(kind=D.WAITALL, req=0, nreq=n))
    r1 = [dict(kind=D.IRECV, peer=0, tag=tag0 + i, count=count, datatype=M.INT32,
               buf=dst.data_ptr() + 4 * count * i, req=i) for i in range(n)]
    r1.append(dict(kind=D.WAITALL, req=0, nreq=n))
    rc, res, _ = sess.run([D.ops_array(r0), D.ops_array(r1)])
    assert rc == 0, M.errname(rc)
    assert torch.equal(src, dst)


def test_trace_records_the_steps_of_every_message_in_order():
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    _say("trace: 16 fused + 16 split messages and one allreduce, 2 ranks")
    sess = D.Session(2, _cfg(trace_events=4096))
    try:
        _messages(D, M, sess, 16, 1024, 0)          # 4 KiB: fused copy
        _messages(D, M, sess, 16, 32768, 100)       # 128 KiB: wait, copy, signal
        a = [torch.full((256,), r + 1, dtype=torch.int32, device="cuda") for r in range(2)]
        b = [torch.zeros(256, dtype=torch.int32, device="cuda") for _ in range(2)]
        torch.cuda.synchronize()
        ops = [D.ops_array([dict(kind=D.ALLREDUCE, count=256, datatype=M.INT32, op=M.SUM,
                                 buf=a[r].data_ptr(), buf2=b[r].data_ptr())]) for r in range(2)]
        rc, _, _ = sess.run(ops)
        assert rc == 0, M.errname(rc)
        assert all(int(x) == 3 for x in b[0].cpu()) and torch.equal(b[0], b[1])
        rc, total, ev = M.mpixs_world_trace(sess.world, 4096)
        assert rc == 0
        assert total == len(ev) == 4 * 32 + 4, (total, len(ev))
        # messages: group by (channel block, value)
        groups = defaultdict(list)
        for e in ev:
            groups[(e.counter & ~63, e.value)].append(e)
        msgs = 0
        for key, es in groups.items():
            kinds = sorted(e.kind for e in es)
            if kinds != [M.TRACE_POST, M.TRACE_MATCH, M.TRACE_DONE, M.TRACE_COMPLETE]:
                continue
            msgs += 1
            k = {e.kind: e for e in es}
            assert k[M.TRACE_POST].counter == k[M.TRACE_MATCH].counter      # the ready word
            assert k[M.TRACE_DONE].counter == k[M.TRACE_COMPLETE].counter   # the done word
            assert k[M.TRACE_POST].counter != k[M.TRACE_DONE].counter
            t = [k[x].time_ns for x in (M.TRACE_POST, M.TRACE_MATCH, M.TRACE_DONE,
                                        M.TRACE_COMPLETE)]
            assert t == sorted(t), (key, t)
            assert k[M.TRACE_MATCH].stream == k[M.TRACE_DONE].stream        # the copier
            assert k[M.TRACE_POST].stream == k[M.TRACE_COMPLETE].stream     # the first side
            assert k[M.TRACE_POST].stream != k[M.TRACE_MATCH].stream
        assert msgs == 32, msgs
        # the allreduce: POST (arrival) and MATCH on the arrive line, DONE and
        # COMPLETE on the done line, the reducing rank's stream in between
        rest = [e for es in groups.values() if len(es) != 4 for e in es]
        rest += [e for es in groups.values() if len(es) == 4 and
                 sorted(x.kind for x in es) != [1, 2, 3, 4] for e in es]
        assert sorted(e.kind for e in rest) == [1, 2, 3, 4], [(e.kind, e.counter, e.value) for e in rest]
        k = {e.kind: e for e in rest}
        assert k[M.TRACE_POST].time_ns <= k[M.TRACE_MATCH].time_ns <= k[M.TRACE_DONE].time_ns \
            <= k[M.TRACE_COMPLETE].time_ns
        assert k[M.TRACE_MATCH].stream == k[M.TRACE_DONE].stream
        assert k[M.TRACE_POST].stream == k[M.TRACE_COMPLETE].stream
    finally:
        torch.cuda.synchronize()
        sess.close()


def test_trace_ring_keeps_the_newest_events_and_is_off_by_default():
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    _say("trace: a ring of 16 events after 40 messages; no trace without the option")
    sess = D.Session(2, _cfg(trace_events=16))
    try:
        _messages(D, M, sess, 40, 256, 0)
        rc, total, ev = M.mpixs_world_trace(sess.world, 100)
        assert rc == 0 and total == 160 and len(ev) == 16
        rc, total, ev = M.mpixs_world_trace(sess.world, 5)
        assert rc == 0 and total == 160 and len(ev) == 5
    finally:
        torch.cuda.synchronize()
        sess.close()
    sess = D.Session(2)
    try:
        _messages(D, M, sess, 2, 256, 0)
        rc, _, _ = M.mpixs_world_trace(sess.world, 10)
        assert M.errname(rc) == "ERR_ARG"
    finally:
        torch.cuda.synchronize()
        sess.close()


def test_trace_of_a_persistent_batch_orders_every_run():
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    n, runs, count = 4, 6, 1024
    _say(f"trace: persistent ring batch, {n} ranks, {runs} runs of 4 KiB messages")
    src = [torch.full((count,), 10 * (r + 1), dtype=torch.int32, device="cuda") for r in range(n)]
    dst = [torch.zeros(count, dtype=torch.int32, device="cuda") for _ in range(n)]
    torch.cuda.synchronize()
    sess = D.Session(n, _cfg(trace_events=4096))
    try:
        ops = []
        for r in range(n):
            rows = [dict(kind=D.GROUP_START),
                    dict(kind=D.ISEND, peer=(r + 1) % n, tag=7, count=count, datatype=M.INT32,
                         buf=src[r].data_ptr(), req=0),
                    dict(kind=D.IRECV, peer=(r - 1) % n, tag=7, count=count, datatype=M.INT32,
                         buf=dst[r].data_ptr(), req=1),
                    dict(kind=D.WAITALL, req=0, nreq=2),
                    dict(kind=D.GROUP_INIT, req=2)]
            rows += [dict(kind=D.BATCH_START, req=2)] * runs
            ops.append(D.ops_array(rows))
        rc, _, _ = sess.run(ops, max_reqs=3)
        assert rc == 0, M.errname(rc)
        for r in range(n):
            assert torch.equal(dst[r], src[(r - 1) % n]), r
        rc, total, ev = M.mpixs_world_trace(sess.world, 4096)
        assert rc == 0 and total == len(ev)
        by = defaultdict(lambda: defaultdict(list))
        for e in ev:
            by[e.value][e.kind].append(e)
        done = sorted(v for v in by if by[v][M.TRACE_DONE])
        assert done == list(range(1, runs + 1)), done
        leader = by[1][M.TRACE_DONE][0].stream
        for v in done:
            k = by[v]
            assert len(k[M.TRACE_DONE]) == 1
            d = k[M.TRACE_DONE][0]
            assert d.stream == leader
            posts = {e.stream: e for e in k[M.TRACE_POST]}
            matches = {e.counter: e for e in k[M.TRACE_MATCH]}
            comps = {e.stream: e for e in k[M.TRACE_COMPLETE]}
            # every other rank arrives once, is seen once, completes once
            assert len(posts) == len(k[M.TRACE_POST]) == n - 1 and leader not in posts
            assert len(matches) == len(k[M.TRACE_MATCH]) == n - 1
            assert all(e.stream == leader for e in k[M.TRACE_MATCH])
            assert set(comps) == set(posts) and len(k[M.TRACE_COMPLETE]) == n - 1
            for s, p in posts.items():
                m = matches[p.counter]                      # the same arrival word
                assert p.time_ns <= m.time_ns <= d.time_ns <= comps[s].time_ns, (v, s)
                assert comps[s].counter == d.counter       # the done word
                if v > 1:
                    assert by[v - 1][M.TRACE_COMPLETE] and \
                        {e.stream: e for e in by[v - 1][M.TRACE_COMPLETE]}[s].time_ns <= p.time_ns
    finally:
        torch.cuda.synchronize()
        sess.close()
