"""Enqueued allreduces read back after per-stream synchronisation only.

The benchmark's grouped-allreduce pattern: 16 ranks, 16 `allreduce_enqueue`
calls per step, each on its own 1 MiB slice of 16 MiB send and receive
buffers, run by the native driver (one host thread per rank, each
synchronising only its own stream at the end).  Before it, a host-
synchronised pass over buffers of the same sizes is run and its buffers are
freed, so the caching allocator hands the same device memory to the
enqueued pass.  Every element of every rank's receive buffer must equal the
oracle's canonical-order float32 fold, read three ways after the rank
streams alone have been synchronised (no device-wide synchronisation): an
on-device comparison, a copy into pinned host memory and a copy into
pageable host memory.  The stream contract of §3.4 needs nothing more.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N = 16
SLICE = 1 << 20
G = 16
STEPS = 20


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _ops(D, M, S, R, count, k):
    out = []
    for r in range(N):
        rows = []
        for _ in range(k):
            rows += [dict(kind=D.ALLREDUCE, count=count, datatype=M.FLOAT32, op=M.SUM,
                          buf=S[r].data_ptr() + i * SLICE, buf2=R[r].data_ptr() + i * SLICE)
                     for i in range(G)]
        out.append(D.ops_array(rows))
    return out


def _run(sess, ops, mode=0):
    from paper_2208_13707_amd import mpixs as M
    rc, res, _ = sess.run(ops, mode=mode)
    assert rc == 0, f"driver: {M.errname(rc)} at thread {res.error_thread} op {res.error_op}"


def _mismatches(R, want_dev, want_np, count):
    """(on-device, pinned, pageable) counts of elements that differ."""
    import torch
    dev = pinned = pageable = 0
    for r in range(N):
        v = R[r].view(torch.int32).view(G, count)
        dev += int((v != want_dev.unsqueeze(0)).sum().item())
        h = torch.empty(R[r].numel(), dtype=torch.uint8, pin_memory=True)
        h.copy_(R[r])
        torch.cuda.current_stream().synchronize()
        pinned += int((h.numpy().view(np.int32).reshape(G, count) != want_np[None, :]).sum())
        pg = R[r].cpu().numpy().view(np.int32).reshape(G, count)
        pageable += int((pg != want_np[None, :]).sum())
    return dev, pinned, pageable


def test_sliced_enqueued_allreduces_after_buffer_reuse_per_stream_sync():
    import torch
    from oracle import reduce as redo
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    from workloads import configs as C

    count = SLICE // 4
    p = C.allreduce(SLICE, "float32", nranks=N, calls=1)
    ins = [np.frombuffer(p.buffers[q]["send"].tobytes(), dtype=np.float32) for q in range(N)]
    # the result's bit patterns, compared as int32 so that every bit counts
    want_np = redo.fold("sum", ins).view(np.int32)
    want_dev = torch.from_numpy(want_np.copy()).cuda()
    base = [torch.from_numpy(p.buffers[r]["send"]).cuda() for r in range(N)]

    _say("[readback] host-synchronised pass over buffers of the same sizes, then freed")
    S0 = [b.repeat(G) for b in base]
    R0 = [torch.zeros(G * SLICE, dtype=torch.uint8, device="cuda") for _ in range(N)]
    torch.cuda.current_stream().synchronize()
    sess = D.Session(N)
    try:
        _run(sess, _ops(D, M, S0, R0, count, 2), mode=1)
        assert _mismatches(R0, want_dev, want_np, count) == (0, 0, 0)
    finally:
        sess.close()
    del S0, R0

    S = [b.repeat(G) for b in base]
    R = [torch.zeros(G * SLICE, dtype=torch.uint8, device="cuda") for _ in range(N)]
    torch.cuda.current_stream().synchronize()
    sess = D.Session(N)
    try:
        for run in range(3):
            _say(f"[readback] enqueue pass {run}: {N} ranks x {G} allreduces x {STEPS} steps")
            _run(sess, _ops(D, M, S, R, count, STEPS))
            # the driver's rank threads synchronised their own streams; nothing else
            got = _mismatches(R, want_dev, want_np, count)
            assert got == (0, 0, 0), f"pass {run}: (device, pinned, pageable) mismatches {got}"
            for t in R:
                t.zero_()
            torch.cuda.current_stream().synchronize()
        assert not any(sess.stream_errors())
    finally:
        sess.close()
