"""Eager sends (§3.4: an enqueue call returns once the operation is
registered), through the C ABI.

A blocking send of at most eager_max_bytes whose receive is not enqueued yet
is packed into device staging on the sender's stream and is complete there,
so the call returns without waiting for its receiver:

* blocking sends of every layout kind (contiguous, vector, irregular
  indexed, odd byte counts, an empty message, a second message on a
  channel) all return before any receive is enqueued, from one host thread,
  under both matching modes (sequence pairing, ordered queues);
  the receives that follow (one truncating, one of another basic type) give
  the oracle's bytes and statuses, and the statistics count every send as
  eager;
* with staging smaller than the messages in flight, the sends beyond it take
  the rendezvous protocol (waiting for their receives), every message still
  arrives, and staging freed by the receives is used again;
* with a matching table of 64 blocks, 1,000 eager messages on 1,000 distinct
  channels run: the receiver's copy, the last device use of each block,
  releases it.
"""
import sys

import numpy as np
import pytest

from oracle import simulate as sim
from tests.gpu_runner import _Types
from workloads.program import Program, Recv, Send

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def _cfg(**kw):
    from paper_2208_13707_amd import mpixs as M
    c = M.Config()
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def _sync_all(sess):
    from paper_2208_13707_amd import driver as D
    lib = D._hiplib()
    lib.hipStreamSynchronize.argtypes = [D.ctypes.c_void_p]
    for hs in sess.hs:
        assert lib.hipStreamSynchronize(hs) == 0


def _close(sess):
    import torch
    torch.cuda.synchronize()
    sess.close()


def _span(tree, count):
    """Bytes from the buffer start that `count` elements of a type touch."""
    from oracle import typemap as tm
    if count == 0:
        return 0
    t = tm.build(tree)
    return (count - 1) * t.extent + t.ub


# (count, send type, receive count, receive type, tag) -- all from rank 0 to 1
IRREG = ("indexed", (3, 1, 4, 1, 5), (0, 5, 7, 13, 20), "float32")
CASES = [
    (1, "int32", 1, "int32", 0),
    (1000, "float32", 1000, "float32", 1),
    (16384, "int32", 16384, "int32", 2),                       # exactly 64 KiB
    (1, ("vector", 2000, 3, 8, "float32"), 1, ("vector", 2000, 3, 8, "float32"), 3),
    (150, IRREG, 150, IRREG, 4),
    (301, "uint8", 301, "uint8", 5),
    (0, "int32", 4, "int32", 6),                               # empty: posts ready only
    (17, "float64", 17, "float64", 0),                         # second message on tag 0
    (200, "int32", 50, "int32", 7),                            # truncated at the receive
    (64, "int32", 64, "float32", 8),                           # other basic type
    (2000, ("vector", 2, 3, 8, "float32"), 12000, "float32", 9),  # vector into contiguous
]


def _program(matching):
    rng = np.random.default_rng(11)
    soff, roff, sends, recvs = 0, 0, [], []
    for i, (sc, st, rc, rt, tag) in enumerate(CASES):
        sends.append(Send("s", soff, sc, st, 1, tag))
        recvs.append(Recv("r", roff, rc, rt, 0, tag, status=f"st{i}"))
        soff += -(-max(1, _span(st, sc)) // 256) * 256
        roff += -(-max(1, _span(rt, rc)) // 256) * 256
    b0 = {"s": rng.integers(0, 256, soff, dtype=np.uint8)}
    b1 = {"r": np.full(roff, 0xEE, np.uint8)}
    return Program(2, [b0, b1], [[sends], [recvs]], 1, name="eager-cases", matching=matching)


@pytest.mark.parametrize("matching", ["sequence", "queue"])
def test_eager_blocking_sends_complete_before_their_receives(matching):
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    _say(f"eager ({matching} matching): {len(CASES)} blocking sends return before any receive; "
         "bytes and statuses vs the oracle")
    p = _program(matching)
    ref = sim.run(p)
    assert not ref.deadlock and not any(ref.sync_errors)
    # a send that waited for its receive would time out here (one thread)
    sess = D.Session(2, _cfg(timeout_ms=5000, matching=1 if matching == "queue" else 0))
    try:
        T = _Types(M)
        s = torch.from_numpy(p.buffers[0]["s"].copy()).cuda()
        r = torch.from_numpy(p.buffers[1]["r"].copy()).cuda()
        sts = torch.zeros(len(CASES) * M.STATUS_BYTES, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        for op in p.ops[0][0]:
            rc = M.mpixs_send_enqueue(s.data_ptr() + op.off, op.count, T.get(op.dtype), op.dest,
                                      op.tag, sess.comms[0])
            assert rc == 0, f"send tag {op.tag}: {M.errname(rc)}"
        for i, op in enumerate(p.ops[1][0]):
            rc = M.mpixs_recv_enqueue(r.data_ptr() + op.off, op.count, T.get(op.dtype), op.source,
                                      op.tag, sess.comms[1], sts.data_ptr() + i * M.STATUS_BYTES)
            assert rc == 0, f"recv tag {op.tag}: {M.errname(rc)}"
        _sync_all(sess)
        assert np.array_equal(r.cpu().numpy(), ref.buffers[1]["r"])
        raw = sts.cpu().numpy().tobytes()
        for i in range(len(CASES)):
            st = M.Status.from_buffer_copy(raw[i * M.STATUS_BYTES:(i + 1) * M.STATUS_BYTES])
            want = ref.statuses[1][f"st{i}"]
            got = (st.source, st.tag, M.errname(st.error) if st.error else "SUCCESS", st.count_bytes)
            assert got == want, f"case {i}: {got} != {want}"
        rc, stats = M.mpixs_world_get_stats(sess.world)
        assert rc == 0
        assert stats.eager_sends == len(CASES)
        for q in range(2):
            rc, e = M.mpixs_stream_get_error(sess.streams[q])
            # the receiver's sticky error is its first failed receive's
            assert rc == 0 and M.errname(e) == ("SUCCESS" if q == 0 else "ERR_TRUNCATE")
    finally:
        _close(sess)


def test_eager_falls_back_when_staging_is_full_and_reuses_it():
    import threading
    import time
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    _say("eager: 1 MiB of staging, 40 blocking sends of 60 KB, receives 0.5 s later, two rounds")
    n, cnt = 40, 15000   # 60,000 bytes of int32 each
    sess = D.Session(2, _cfg(eager_arena_mib=1, timeout_ms=20000))
    try:
        src = torch.arange(n * cnt, dtype=torch.int32, device="cuda")
        dst = torch.zeros(n * cnt, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        seen = 0
        for rnd in range(2):
            dst.zero_()
            torch.cuda.synchronize()
            errs = []

            def receiver():
                time.sleep(0.5)
                for i in range(n):
                    rc = M.mpixs_recv_enqueue(dst.data_ptr() + 4 * cnt * i, cnt, M.INT32, 0,
                                              100 * rnd + i, sess.comms[1])
                    if rc:
                        errs.append(f"recv {i}: {M.errname(rc)}")
                        return

            th = threading.Thread(target=receiver)
            th.start()
            for i in range(n):
                rc = M.mpixs_send_enqueue(src.data_ptr() + 4 * cnt * i, cnt, M.INT32, 1,
                                          100 * rnd + i, sess.comms[0])
                assert rc == 0, f"send {i}: {M.errname(rc)}"
            th.join(60)
            assert not th.is_alive() and not errs, errs
            _sync_all(sess)
            assert torch.equal(src, dst), f"round {rnd}"
            rc, stats = M.mpixs_world_get_stats(sess.world)
            eager = stats.eager_sends - seen
            seen = stats.eager_sends
            # 1 MiB holds 17 slots of 60,000 bytes (256-byte aligned); the
            # 18th send waits for its receive, after which the others may find
            # their receives enqueued already
            assert 1 <= eager < n, f"round {rnd}: {eager} eager sends"
    finally:
        _close(sess)


def test_eager_messages_release_their_channel_blocks():
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    _say("eager: 1,000 messages on distinct channels with a 64-block matching table")
    n = 1000
    sess = D.Session(2, _cfg(max_channels=64, timeout_ms=20000))
    try:
        src = torch.arange(n * 16, dtype=torch.int64, device="cuda")
        dst = torch.zeros(n * 16, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        for i in range(n):
            rc = M.mpixs_send_enqueue(src.data_ptr() + 128 * i, 16, M.INT64, 1, i, sess.comms[0])
            assert rc == 0, f"send {i}: {M.errname(rc)}"
            rc = M.mpixs_recv_enqueue(dst.data_ptr() + 128 * i, 16, M.INT64, 0, i, sess.comms[1])
            assert rc == 0, f"recv {i}: {M.errname(rc)}"
        _sync_all(sess)
        assert torch.equal(src, dst)
        rc, stats = M.mpixs_world_get_stats(sess.world)
        assert stats.eager_sends == n
        assert stats.channels_recycled >= n - 64
    finally:
        _close(sess)
