"""The copy kernels' address maps, planned on the host, against the oracle
(CPU only).

For a matched message the library chooses a unit size and two maps from
packed unit index to byte address.  Expanding every unit to its bytes must
give exactly the oracle's pack positions on the sending side and unpack
positions on the receiving side, for the bytes the message moves.  This is
also the bounds check of the copy kernels: no unit reaches outside its
typemap.
"""
import ctypes
import os

import numpy as np
import pytest

from oracle import typemap as tm
from tests.test_host_types import _build
from workloads import configs as C
from workloads.program import Recv, Send

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2208_13707_amd", "libmpixs.so")


@pytest.fixture(scope="module")
def M():
    if not os.path.exists(LIB):
        pytest.fail("libmpixs.so is not built")
    from paper_2208_13707_amd import mpixs as M
    f = M.lib().mpixs_debug_copy_plan
    f.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int,
                  ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                  ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64)]
    f.restype = ctypes.c_int
    return M


def plan(M, sbuf, scount, stree, rbuf, rcount, rtree, nbytes):
    rc, st = _build(M, stree)
    assert rc == 0
    rc, rt = _build(M, rtree)
    assert rc == 0
    n_max = nbytes  # units never exceed bytes
    src = np.zeros(max(n_max, 1), np.uint64)
    dst = np.zeros(max(n_max, 1), np.uint64)
    w = ctypes.c_int()
    n = ctypes.c_int64()
    P = ctypes.POINTER(ctypes.c_uint64)
    rc = M.lib().mpixs_debug_copy_plan(sbuf, scount, st, rbuf, rcount, rt, nbytes, n_max,
                                       src.ctypes.data_as(P), dst.ctypes.data_as(P),
                                       ctypes.byref(w), ctypes.byref(n))
    assert rc == 0
    return w.value, n.value, src[: n.value].astype(np.int64), dst[: n.value].astype(np.int64)


def check(M, stree, scount, soff, rtree, rcount, roff, base=1 << 20):
    ts, tr = tm.build(stree), tm.build(rtree)
    assert ts.basic == tr.basic
    nbytes = min(scount * ts.size, rcount * tr.size)
    w, n, src, dst = plan(M, base + soff, scount, stree, (base << 4) + roff, rcount, rtree, nbytes)
    assert w in (1, 2, 4, 8, 16) and n * w == nbytes
    want_s = tm.byte_positions(ts, scount, base + soff)[:nbytes]
    want_r = tm.byte_positions(tr, rcount, (base << 4) + roff)[:nbytes]
    got_s = (src[:, None] + np.arange(w)[None, :]).reshape(-1)
    got_r = (dst[:, None] + np.arange(w)[None, :]).reshape(-1)
    assert np.array_equal(got_s, want_s)
    assert np.array_equal(got_r, want_r)
    for a in (src, dst):   # every unit is aligned to its size
        assert np.all(a % w == 0)
    return w


def test_halo_vector_uses_4_byte_units(M):
    vt = C.halo_type(43690)
    assert check(M, vt, 1, 0, vt, 1, 0) == 4
    assert check(M, vt, 1, 12, vt, 1, 12) == 4


def test_contiguous_uses_16_byte_units(M):
    assert check(M, "int32", 1024, 0, "int32", 1024, 0) == 16
    assert check(M, "int32", 1023, 0, "int32", 1024, 0) == 4     # 4092 bytes
    assert check(M, "uint8", 4096, 3, "uint8", 4096, 0) == 1


CASES = [
    (("vector", 5, 3, 8, "float32"), 2, 0, "float32", 40, 0),
    ("float32", 40, 4, ("vector", 5, 3, 8, "float32"), 2, 8),
    (("indexed", [3, 1, 4, 2], [0, 5, 7, 13], "int32"), 3, 0,
     ("vector", 10, 3, 5, "int32"), 3, 4),
    (("contiguous", 2, ("vector", 3, 1, 3, "int32")), 4, 0, "int32", 24, 0),
    (("vector", 2, 2, 3, ("indexed", [2], [5], "float32")), 3, 0,
     ("indexed", [2], [5], "float32"), 12, 0),
    (("vector", 3, 2, 7, "float64"), 5, 8, ("vector", 6, 5, 9, "float64"), 1, 0),
    (("indexed", [1, 2], [3, 0], "int8"), 7, 1, "int8", 21, 2),
    (("vector", 4, 4, 4, "int64"), 2, 0, "int64", 32, 8),
    (("vector", 1000, 2, 5, "int32"), 1, 0, ("vector", 500, 4, 9, "int32"), 1, 0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: str(c[0])[:40])
def test_mixed_layouts(M, case):
    check(M, *case)


def test_truncated_message_plan(M):
    # the receiver holds fewer bytes: only its capacity is planned
    check(M, ("vector", 9, 3, 8, "float32"), 1, 0, "float32", 20, 0)


@pytest.mark.parametrize("seed", range(6))
def test_random_program_messages(M, seed):
    p = C.random_program(seed)
    sends, recvs = {}, {}
    for r in range(p.nranks):
        for o in p.ops[r][0]:
            if isinstance(o, Send):
                sends[o.req[1:]] = o
            elif isinstance(o, Recv):
                recvs[o.req[1:]] = o
    for key, s in sends.items():
        r = recvs[key]
        check(M, s.dtype, s.count, s.off, r.dtype, r.count, r.off)


@pytest.mark.parametrize("i", range(40))
def test_batch_messages(M, i):
    m = C.batch_messages(npairs=40)[i]
    check(M, m["tree"], m["count"], 256 * (i % 3), m["tree"], m["count"], 512 * (i % 2))
