"""Messages at the size limits, through the C ABI.

* A contiguous message of 4,295,012,885 bytes (above 2^32, a ragged byte
  count): 64-bit offsets in the copy and batch kernels and the batch
  kernel's byte tail.
* A vector message of 2^32 - 1 one-byte units, the most a non-dense layout
  may carry (its unit index is 32-bit on the device): every unit index up to
  the limit.
* One more element of the vector type is refused at once (ERR_COUNT) and
  leaves no trace on the channel.

The expected result of a copy is its definition: the receive buffer's packed
bytes equal the send buffer's packed bytes.  Both buffers stay on the device
and are compared there, element by element, on the full message.
"""
import sys

import pytest

pytestmark = pytest.mark.gpu

CONTIG_ELEM = 1_000_003          # bytes per element of the contiguous type
CONTIG_COUNT = 4295              # 4,295,012,885 bytes
VEC_BLOCKS = 65535               # vector(65535, 1, 2, uint8): size 65535, extent 131069
VEC_COUNT = 65537                # 65535 * 65537 = 2^32 - 1 bytes


def _say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def _types(M):
    rc, tc = M.mpixs_type_contiguous(CONTIG_ELEM, M.UINT8)
    assert rc == 0
    rc, tc = M.mpixs_type_commit(tc)
    assert rc == 0
    rc, tv = M.mpixs_type_vector(VEC_BLOCKS, 1, 2, M.UINT8)
    assert rc == 0
    rc, tv = M.mpixs_type_commit(tv)
    assert rc == 0
    rc, tr = M.mpixs_type_contiguous(VEC_BLOCKS, M.UINT8)
    assert rc == 0
    rc, tr = M.mpixs_type_commit(tr)
    assert rc == 0
    return tc, tv, tr


def _run(sess, D, M, rows0, rows1, mode=0):
    rc, res, _ = sess.run([D.ops_array(rows0), D.ops_array(rows1)], mode=mode)
    assert rc == 0, f"{M.errname(rc)} at thread {res.error_thread} op {res.error_op}"
    assert sess.stream_errors() == [0, 0]


def _pair(D, send, recv, grouped):
    if not grouped:
        return [send], [recv]
    return ([dict(kind=D.GROUP_START), send, dict(kind=D.GROUP_END)],
            [dict(kind=D.GROUP_START), recv, dict(kind=D.GROUP_END)])


@pytest.mark.parametrize("path", ["enqueue", "grouped", "host-synced"])
def test_contiguous_message_above_4gib(path):
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    n = CONTIG_ELEM * CONTIG_COUNT
    _say(f"contiguous {n} bytes, {path}")
    g = torch.Generator(device="cuda").manual_seed(20813707)
    src = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.zeros(n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    sess = D.Session(2)
    try:
        tc, _, _ = _types(M)
        send = dict(kind=D.SEND, peer=1, tag=5, count=CONTIG_COUNT, datatype=tc, buf=src.data_ptr())
        recv = dict(kind=D.RECV, peer=0, tag=5, count=CONTIG_COUNT, datatype=tc, buf=dst.data_ptr())
        r0, r1 = _pair(D, send, recv, path == "grouped")
        _run(sess, D, M, r0, r1, mode=1 if path == "host-synced" else 0)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)
    finally:
        sess.close()
        del src, dst
        torch.cuda.empty_cache()


@pytest.mark.parametrize("grouped", [False, True])
def test_vector_message_at_the_unit_limit(grouped):
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    ext = 2 * VEC_BLOCKS - 1
    _say(f"vector {VEC_COUNT} x vector({VEC_BLOCKS}, 1, 2, uint8), grouped={grouped}")
    g = torch.Generator(device="cuda").manual_seed(2208)
    src = torch.randint(0, 256, (VEC_COUNT * ext,), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.zeros(VEC_COUNT * VEC_BLOCKS, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    sess = D.Session(2)
    try:
        _, tv, tr = _types(M)
        send = dict(kind=D.SEND, peer=1, tag=9, count=VEC_COUNT, datatype=tv, buf=src.data_ptr())
        recv = dict(kind=D.RECV, peer=0, tag=9, count=VEC_COUNT, datatype=tr, buf=dst.data_ptr())
        r0, r1 = _pair(D, send, recv, grouped)
        _run(sess, D, M, r0, r1)
        torch.cuda.synchronize()
        # element k of the send starts at k * extent; block j at 2j within it
        want = src.view(VEC_COUNT, ext)[:, ::2]
        assert want.shape == (VEC_COUNT, VEC_BLOCKS)
        assert torch.equal(dst.view(VEC_COUNT, VEC_BLOCKS), want)
    finally:
        sess.close()
        del src, dst
        torch.cuda.empty_cache()


def test_vector_message_beyond_the_unit_limit_is_refused():
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    _say("vector beyond the unit limit: ERR_COUNT without side effects")
    a = torch.arange(64, dtype=torch.uint8, device="cuda")
    b = torch.zeros(64, dtype=torch.uint8, device="cuda")
    sess = D.Session(2)
    try:
        _, tv, _ = _types(M)
        # 65538 elements of 65535 bytes: 2^32 + 65534 bytes of a non-dense
        # layout, refused before anything is enqueued or any buffer read
        rc = M.mpixs_send_enqueue(a, VEC_COUNT + 1, tv, 1, 3, sess.comms[0])
        assert M.errname(rc) == "ERR_COUNT"
        # the channel is untouched: the next send on it is message 0
        send = dict(kind=D.SEND, peer=1, tag=3, count=64, datatype=M.UINT8, buf=a.data_ptr())
        recv = dict(kind=D.RECV, peer=0, tag=3, count=64, datatype=M.UINT8, buf=b.data_ptr())
        _run(sess, D, M, [send], [recv])
        torch.cuda.synchronize()
        assert torch.equal(a, b)
    finally:
        sess.close()
