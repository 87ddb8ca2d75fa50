"""Finite resources and the boundary's refusals, through the C ABI (§3.1, §6).

* Endpoints are finite (§2.2, §3.1): stream creation fails with
  ERR_NO_ENDPOINT once the pool is empty (policy 0) and succeeds again after
  a free; under policy 1 streams share endpoints round-robin, and a program
  run on more streams than endpoints still equals the oracle.
* MPIX_Stream_free may fail (§3.1): ERR_PENDING while a communicator uses
  the stream or while work enqueued on it has not finished; the stream stays
  valid and its free succeeds once the stream is idle.
* Frees return resources (§3.1): with a matching table of 64 blocks,
  10,000 messages on 10,000 distinct channels run in both matching modes
  (sequence pairing, ordered queues) and equal the oracle; 2,000 cycles of
  stream and communicator creation and free (each with a message and an
  allreduce) run on a world whose stream and collective pools hold far
  fewer; the statistics count the recycled blocks.
* Buffers must be GPU-accessible (§6's GPU example sends host memory): a
  pageable host buffer or status, or bytes beyond the buffer's allocation,
  is ERR_BUFFER at the call with no side effect; a status in pinned host
  memory is accepted.
"""
import struct
import sys
import threading

import numpy as np
import pytest

from oracle import reduce as redo
from oracle import simulate as sim
from tests.gpu_runner import compare, run_program
from workloads import configs as C
from workloads.program import Program, Recv, Send, Wait, as_bytes

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def _cfg(**kw):
    from paper_2208_13707_amd import mpixs as M
    c = M.Config()
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def _hip_stream():
    from paper_2208_13707_amd import driver as D
    return D.hip_stream_create()


def _stream(M, world, hs):
    rc, info = M.mpixs_info_create()
    assert rc == 0
    M.mpixs_info_set(info, "type", "hipStream_t")
    M.mpixs_info_set_hex(info, "value", struct.pack("<Q", hs))
    rc, s = M.mpixs_stream_create(world, info)
    M.mpixs_info_free(info)
    return rc, s


def _sync(hs):
    from paper_2208_13707_amd import driver as D
    lib = D._hiplib()
    lib.hipStreamSynchronize.argtypes = [D.ctypes.c_void_p]
    assert lib.hipStreamSynchronize(hs) == 0


# ------------------------------------------------------------ endpoints (§3.1)
def test_endpoint_pool_exhaustion_and_free():
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    _say("endpoint pool of 2: third stream is ERR_NO_ENDPOINT, free makes room")
    rc, w = M.mpixs_world_create(1, _cfg(max_streams=2))
    assert rc == 0
    hs = [_hip_stream() for _ in range(3)]
    try:
        rc0, s0 = _stream(M, w, hs[0])
        rc1, s1 = _stream(M, w, hs[1])
        assert (rc0, rc1) == (0, 0)
        rc2, s2 = _stream(M, w, hs[2])
        assert M.errname(rc2) == "ERR_NO_ENDPOINT" and not s2
        assert M.mpixs_stream_free(s1) == 0
        rc2, s2 = _stream(M, w, hs[2])
        assert rc2 == 0
        assert M.mpixs_stream_free(s2) == 0
        assert M.mpixs_stream_free(s0) == 0
    finally:
        assert M.mpixs_world_free(w) == 0
        for h in hs:
            D.hip_stream_destroy(h)


def test_round_robin_endpoints_parity():
    _say("policy 1: 8 ranks' streams on 3 endpoints, ring halo equals the oracle")
    p = C.ring_halo(count=331, steps=3, update=True)
    ref = sim.run(p)
    g = run_program(p, cfg=_cfg(max_streams=3, endpoint_policy=1))
    diffs = compare(p, g, ref)
    assert not diffs, "\n".join(diffs[:20])


def test_round_robin_off_refuses_more_streams_than_endpoints():
    _say("policy 0: 8 ranks on 3 endpoints cannot set up")
    p = C.ring_halo(count=31, steps=1)
    with pytest.raises(RuntimeError, match="NO_ENDPOINT"):
        run_program(p, cfg=_cfg(max_streams=3, endpoint_policy=0, timeout_ms=2000),
                    timeout_s=20.0)


# ------------------------------------------------------------- stream_free
def test_stream_free_pending_then_success():
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    _say("stream_free: ERR_PENDING with a communicator, then with work in flight")
    rc, w = M.mpixs_world_create(1, None)
    assert rc == 0
    hs = _hip_stream()
    try:
        rc, s = _stream(M, w, hs)
        assert rc == 0
        rc, wc = M.mpixs_world_comm(w, 0)
        rc, c = M.mpixs_comm_create_with_stream(wc, s)
        assert rc == 0
        assert M.errname(M.mpixs_stream_free(s)) == "ERR_PENDING"
        assert M.mpixs_comm_free(c) == 0
        # work in flight on the HIP stream: a spin kernel of a few hundred ms
        ts = torch.cuda.ExternalStream(hs)
        with torch.cuda.stream(ts):
            torch.cuda._sleep(600_000_000)
        assert M.errname(M.mpixs_stream_free(s)) == "ERR_PENDING"
        ts.synchronize()
        assert M.mpixs_stream_free(s) == 0
    finally:
        assert M.mpixs_world_free(w) == 0
        D.hip_stream_destroy(hs)


def test_stream_free_pending_while_a_receive_waits_on_the_device():
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    _say("stream_free: ERR_PENDING while the stream waits for a peer's copy")
    sess = D.Session(2)
    try:
        a = torch.arange(256, dtype=torch.int32, device="cuda")
        b = torch.zeros(256, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        # rank 0's stream is busy first, so its copy (it arrives second)
        # starts late and rank 1's stream waits on the device meanwhile
        t0 = torch.cuda.ExternalStream(sess.hs[0])
        with torch.cuda.stream(t0):
            torch.cuda._sleep(600_000_000)
        rc, rq = M.mpixs_irecv_enqueue(b, 256, M.INT32, 0, 7, sess.comms[1])
        assert rc == 0
        assert M.mpixs_send_enqueue(a, 256, M.INT32, 1, 7, sess.comms[0]) == 0
        rc, _ = M.mpixs_wait_enqueue(rq, None)
        assert rc == 0
        assert M.mpixs_comm_free(sess.comms[1]) == 0
        sess.comms[1] = None
        assert M.errname(M.mpixs_stream_free(sess.streams[1])) == "ERR_PENDING"
        _sync(sess.hs[0])
        _sync(sess.hs[1])
        assert torch.equal(a, b)
        assert M.mpixs_stream_free(sess.streams[1]) == 0
        sess.streams[1] = None
    finally:
        torch.cuda.synchronize()
        for r in range(2):
            if sess.comms[r]:
                M.mpixs_comm_free(sess.comms[r])
            if sess.streams[r]:
                M.mpixs_stream_free(sess.streams[r])
        M.mpixs_world_free(sess.world)
        for h in sess.hs:
            D.hip_stream_destroy(h)


# ---------------------------------------------------- channel block recycling
def _many_channel_program(nmsg, window, matching):
    rng = np.random.default_rng([220813707, 90, nmsg])
    vals = rng.integers(-2**62, 2**62, size=nmsg, dtype=np.int64)
    b0 = {"s": as_bytes(vals)}
    b1 = {"r": np.zeros(8 * nmsg, np.uint8)}
    r0, r1 = [], []
    for w0 in range(0, nmsg, window):
        idx = range(w0, min(nmsg, w0 + window))
        if (w0 // window) % 5 == 4:
            # blocking calls now and then (their waits release at once)
            for i in idx:
                r0.append(Send("s", 8 * i, 1, "int64", 1, i))
                r1.append(Recv("r", 8 * i, 1, "int64", 0, i))
            continue
        for i in idx:
            r0.append(Send("s", 8 * i, 1, "int64", 1, i, req=f"s{i}"))
            r1.append(Recv("r", 8 * i, 1, "int64", 0, i, req=f"r{i}"))
        r0.append(Wait([f"s{i}" for i in idx], [None] * len(idx)))
        r1.append(Wait([f"r{i}" for i in idx], [None] * len(idx)))
    return Program(2, [b0, b1], [[r0], [r1]], 1, [[0, 0]],
                   name=f"{nmsg} messages on distinct channels ({matching})", matching=matching)


@pytest.mark.parametrize("matching", ["sequence", "queue"])
def test_channel_blocks_recycled(matching):
    p = _many_channel_program(10000, 16, matching)
    _say(p.name + ", 64 matching-table blocks")
    ref = sim.run(p)
    assert not ref.deadlock
    g = run_program(p, cfg=_cfg(max_channels=64), stats=True)
    diffs = compare(p, g, ref)
    assert not diffs, "\n".join(diffs[:20])
    assert g.stats.channels_recycled >= 10000 - 64


# ------------------------------------------- stream and communicator cycles
def test_stream_and_communicator_cycles():
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    cycles = 2000
    _say(f"{cycles} cycles of stream + communicator create / message / allreduce / free")
    rng = np.random.default_rng([220813707, 91])
    xs = rng.integers(-2**40, 2**40, size=cycles, dtype=np.int64)
    ins = [rng.integers(-2**40, 2**40, size=cycles, dtype=np.int64) for _ in range(2)]
    x = torch.from_numpy(xs).cuda()
    rbuf = torch.zeros(cycles, dtype=torch.int64, device="cuda")
    ain = [torch.from_numpy(v).cuda() for v in ins]
    aout = [torch.zeros(cycles, dtype=torch.int64, device="cuda") for _ in range(2)]
    torch.cuda.synchronize()
    rc, w = M.mpixs_world_create(2, _cfg(max_streams=4, max_collectives=64))
    assert rc == 0
    hs = [_hip_stream() for _ in range(2)]
    bar = threading.Barrier(2)
    errs = []

    def rank(r):
        try:
            rc, wc = M.mpixs_world_comm(w, r)
            for cyc in range(cycles):
                rc, s = _stream(M, w, hs[r])
                assert rc == 0, f"cycle {cyc}: stream_create {M.errname(rc)}"
                rc, c = M.mpixs_comm_create_with_stream(wc, s)
                assert rc == 0, f"cycle {cyc}: comm_create {M.errname(rc)}"
                if r == 0:
                    rc = M.mpixs_send_enqueue(x.data_ptr() + 8 * cyc, 1, M.INT64, 1, cyc % 7, c)
                else:
                    rc = M.mpixs_recv_enqueue(rbuf.data_ptr() + 8 * cyc, 1, M.INT64, 0, cyc % 7, c)
                assert rc == 0, f"cycle {cyc}: p2p {M.errname(rc)}"
                rc = M.mpixs_allreduce_enqueue(ain[r].data_ptr() + 8 * cyc,
                                               aout[r].data_ptr() + 8 * cyc, 1, M.INT64, M.SUM, c)
                assert rc == 0, f"cycle {cyc}: allreduce {M.errname(rc)}"
                assert M.mpixs_comm_free(c) == 0
                _sync(hs[r])
                rc, e = M.mpixs_stream_get_error(s)
                assert rc == 0 and e == 0, f"cycle {cyc}: stream error {M.errname(e)}"
                assert M.mpixs_stream_free(s) == 0
                bar.wait(timeout=60)
        except Exception as ex:  # reported below
            errs.append(repr(ex))
            bar.abort()

    th = [threading.Thread(target=rank, args=(r,)) for r in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(300)
    try:
        assert not errs, errs
        rc, st = M.mpixs_world_get_stats(w)
        assert rc == 0
        assert st.streams_recycled >= 2 * cycles - 1024
        assert st.comm_lines_recycled >= cycles - 64 * 16 // (2 * 16 * 3)
        assert np.array_equal(rbuf.cpu().numpy(), xs)
        want = redo.fold("sum", ins)
        for r in range(2):
            assert np.array_equal(aout[r].cpu().numpy(), want)
    finally:
        assert M.mpixs_world_free(w) == 0
        for h in hs:
            D.hip_stream_destroy(h)


# ------------------------------------------------------- buffers (ERR_BUFFER)
def test_pageable_host_buffer_is_refused_without_side_effects():
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    _say("ERR_BUFFER: pageable host send buffer, then the channel's message 0 moves")
    host = np.arange(64, dtype=np.int32)
    a = torch.arange(64, dtype=torch.int32, device="cuda")
    b = torch.zeros(64, dtype=torch.int32, device="cuda")
    sess = D.Session(2, _cfg(timeout_ms=5000))
    try:
        # a sender-only call: no receive is posted, so nothing would touch
        # the buffer even if the check were missing
        rc, rq = M.mpixs_isend_enqueue(host.ctypes.data, 64, M.INT32, 1, 3, sess.comms[0])
        assert M.errname(rc) == "ERR_BUFFER" and not rq
        rc, rq = M.mpixs_isend_enqueue(torch.zeros(4).data_ptr(), 4, M.FLOAT32, 1, 3, sess.comms[0])
        assert M.errname(rc) == "ERR_BUFFER" and not rq
        send = dict(kind=D.SEND, peer=1, tag=3, count=64, datatype=M.INT32, buf=a.data_ptr())
        recv = dict(kind=D.RECV, peer=0, tag=3, count=64, datatype=M.INT32, buf=b.data_ptr())
        rc, res, _ = sess.run([D.ops_array([send]), D.ops_array([recv])])
        assert rc == 0
        assert torch.equal(a, b)
        assert not any(sess.stream_errors())
    finally:
        sess.close()


def test_bytes_beyond_the_allocation_are_refused():
    import ctypes
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    _say("ERR_BUFFER: a message running past the end of its allocation")
    lib = D._hiplib()
    lib.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    lib.hipFree.argtypes = [ctypes.c_void_p]
    lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    size = 2 << 20
    base = ctypes.c_void_p()
    assert lib.hipMalloc(ctypes.byref(base), size) == 0   # an allocation of its own
    sess = D.Session(2, _cfg(timeout_ms=5000))
    vt = None
    try:
        end = base.value + size
        rc, rq = M.mpixs_isend_enqueue(end - 1024, 2048, M.UINT8, 1, 5, sess.comms[0])
        assert M.errname(rc) == "ERR_BUFFER" and not rq
        # a vector type whose last block ends past the allocation
        rc, vt = M.mpixs_type_vector(2, 1, 4096, M.UINT8)
        assert rc == 0
        rc, vt = M.mpixs_type_commit(vt)
        assert rc == 0
        rc, rq = M.mpixs_isend_enqueue(end - 4096, 1, vt, 1, 5, sess.comms[0])
        assert M.errname(rc) == "ERR_BUFFER" and not rq
        # ending at the allocation's last byte is fine
        one = np.array([11], np.uint8)
        two = np.array([22], np.uint8)
        assert lib.hipMemcpy(end - 4097, one.ctypes.data, 1, 1) == 0   # host to device
        assert lib.hipMemcpy(end - 1, two.ctypes.data, 1, 1) == 0
        rc, rq = M.mpixs_isend_enqueue(end - 4097, 1, vt, 1, 5, sess.comms[0])
        assert rc == 0
        dst = torch.zeros(2, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        assert M.mpixs_recv_enqueue(dst, 2, M.UINT8, 0, 5, sess.comms[1]) == 0
        rc, _ = M.mpixs_wait_enqueue(rq, None)
        assert rc == 0
        _sync(sess.hs[0])
        _sync(sess.hs[1])
        assert dst.tolist() == [11, 22]
    finally:
        sess.close()
        if vt:
            M.mpixs_type_free(vt)
        lib.hipFree(base)


def test_status_in_pageable_host_memory_is_refused_pinned_accepted():
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    _say("ERR_BUFFER: pageable status refused, pinned status written by the device")
    a = torch.arange(32, dtype=torch.int64, device="cuda")
    b = torch.zeros(32, dtype=torch.int64, device="cuda")
    sess = D.Session(2, _cfg(timeout_ms=5000))
    try:
        st_host = np.zeros(M.STATUS_BYTES, np.uint8)
        rc = M.mpixs_recv_enqueue(b, 32, M.INT64, 0, 9, sess.comms[1], st_host.ctypes.data)
        assert M.errname(rc) == "ERR_BUFFER"
        rc, rq = M.mpixs_irecv_enqueue(b, 32, M.INT64, 0, 9, sess.comms[1])
        assert rc == 0
        rc, _ = M.mpixs_wait_enqueue(rq, st_host.ctypes.data)
        assert M.errname(rc) == "ERR_BUFFER"
        pinned = torch.zeros(M.STATUS_BYTES, dtype=torch.uint8, pin_memory=True)
        assert M.mpixs_send_enqueue(a, 32, M.INT64, 1, 9, sess.comms[0]) == 0
        rc, _ = M.mpixs_wait_enqueue(rq, pinned.data_ptr())
        assert rc == 0
        _sync(sess.hs[1])
        src, tag, err, sidx, cnt = struct.unpack("<iiiiq", pinned.numpy().tobytes())
        assert (src, tag, err, cnt) == (0, 9, 0, 256)
        assert torch.equal(a, b)
    finally:
        sess.close()


def test_allreduce_with_a_host_buffer_is_refused_without_side_effects():
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    _say("ERR_BUFFER: allreduce with a pageable receive buffer, then instance 0 runs")
    n = 4
    ins = [np.arange(100, dtype=np.int64) * (r + 1) for r in range(n)]
    dev_in = [torch.from_numpy(v).cuda() for v in ins]
    out = [torch.zeros(100, dtype=torch.int64, device="cuda") for _ in range(n)]
    torch.cuda.synchronize()
    host = np.zeros(100, np.int64)
    sess = D.Session(n, _cfg(timeout_ms=5000))
    try:
        rc = M.mpixs_allreduce_enqueue(dev_in[0], host.ctypes.data, 100, M.INT64, M.SUM,
                                       sess.comms[0])
        assert M.errname(rc) == "ERR_BUFFER"
        ops = [D.ops_array([dict(kind=D.ALLREDUCE, count=100, datatype=M.INT64, op=M.SUM,
                                 buf=dev_in[r].data_ptr(), buf2=out[r].data_ptr())])
               for r in range(n)]
        rc, res, _ = sess.run(ops)
        assert rc == 0
        want = redo.fold("sum", ins)
        for r in range(n):
            assert np.array_equal(out[r].cpu().numpy(), want)
    finally:
        sess.close()
