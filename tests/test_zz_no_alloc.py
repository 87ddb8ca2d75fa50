"""mpixs_group_end_init_static (no device allocation) against
mpixs_group_end_init, through the C ABI.

The same persistent batches (the batch workload's recipe over 8 ranks:
uneven sizes, tags, 30 % vector datatypes) are made both ways and started
twice; every received byte of the static plan's runs must equal those of
the allocated plan's runs.  Two static plans are made in a row, the second
of a smaller group; the first then refuses to start (its region now holds
the second plan).  A plan larger than the static region is refused on every
rank.
"""
import sys

import numpy as np
import pytest

from workloads import configs as C
from workloads.program import Recv, Send, Wait

pytestmark = pytest.mark.gpu

N = 8


def _say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def _group_rows(D, M, p, r, S, R, init_kind, slot, types):
    def tt(tree):
        key = repr(tree)
        if key not in types:
            if isinstance(tree, str):
                types[key] = M.BASIC[tree]
            else:
                _, c, bl, st, base = tree
                rc, t = M.mpixs_type_vector(c, bl, st, M.BASIC[base])
                assert rc == 0
                rc, t = M.mpixs_type_commit(t)
                assert rc == 0
                types[key] = t
        return types[key]

    rows = [dict(kind=D.GROUP_START)]
    nreq = 0
    for o in p.ops[r][0]:
        if isinstance(o, Send):
            rows.append(dict(kind=D.ISEND, peer=o.dest, tag=o.tag, count=o.count,
                             datatype=tt(o.dtype), buf=S[r].data_ptr() + o.off, req=nreq))
            nreq += 1
        elif isinstance(o, Recv):
            rows.append(dict(kind=D.IRECV, peer=o.source, tag=o.tag, count=o.count,
                             datatype=tt(o.dtype), buf=R[r].data_ptr() + o.off, req=nreq))
            nreq += 1
        elif isinstance(o, Wait):
            rows.append(dict(kind=D.WAITALL, req=0, nreq=nreq))
    rows.append(dict(kind=init_kind, req=slot))
    return rows


def _make_and_run(sess, D, M, p, S, R, init_kind, slot, runs, types):
    import torch
    ops = [D.ops_array(_group_rows(D, M, p, r, S, R, init_kind, slot, types)
                       + [dict(kind=D.BATCH_START, req=slot)] * runs) for r in range(N)]
    rc, res, _ = sess.run(ops, max_reqs=max(len(p.ops[r][0]) for r in range(N)) + 1)
    return rc, [x.cpu().numpy().copy() for x in R] if rc == 0 else None


def _bufs(p):
    import torch
    S = [torch.from_numpy(p.buffers[r]["sbuf"]).cuda() for r in range(N)]
    Ra = [torch.from_numpy(p.buffers[r]["rbuf"].copy()).cuda() for r in range(N)]
    Rb = [torch.from_numpy(p.buffers[r]["rbuf"].copy()).cuda() for r in range(N)]
    torch.cuda.synchronize()
    return S, Ra, Rb


def test_static_plan_equals_allocated_plan_two_calls():
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    sess = D.Session(N)
    types = {}
    try:
        for step, npairs in enumerate((4000, 500)):
            p = C.batch(npairs=npairs, nranks=N)
            S, Ra, Rb = _bufs(p)
            _say(f"static plan {step}: {npairs} messages, 8 ranks, against the allocated plan")
            rc, want = _make_and_run(sess, D, M, p, S, Ra, D.GROUP_INIT, 2 * step, 2, types)
            assert rc == 0, M.errname(rc)
            rc, got = _make_and_run(sess, D, M, p, S, Rb, D.GROUP_INIT_STATIC, 2 * step + 1, 2,
                                    types)
            assert rc == 0, M.errname(rc)
            for r in range(N):
                assert np.array_equal(got[r], want[r]), f"plan {step} rank {r}"
                # the runs really moved the messages
                assert not np.array_equal(got[r], p.buffers[r]["rbuf"]) or got[r].size <= 1
        # the first static plan's region now holds the second plan
        for r in range(N):
            assert M.errname(M.mpixs_batch_start_enqueue(sess.batches[r][1])) == "ERR_REQUEST"
    finally:
        sess.close()
        for t in types.values():
            if t > M.FLOAT64:
                M.mpixs_type_free(t)


def test_static_plan_beyond_the_region_is_refused():
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    # 20,000 messages need 224 B each: more than the 4 MiB region
    p = C.batch(npairs=20000, nranks=N, max_bytes=16)
    S, Ra, _ = _bufs(p)
    _say("static plan of 20,000 messages: ERR_NOMEM on every rank")
    sess = D.Session(N)
    types = {}
    try:
        rc, _ = _make_and_run(sess, D, M, p, S, Ra, D.GROUP_INIT_STATIC, 0, 0, types)
        assert M.errname(rc) == "ERR_NOMEM"
        assert all(not sess.batches[r][0] for r in range(N))
    finally:
        sess.close()
        for t in types.values():
            if t > M.FLOAT64:
                M.mpixs_type_free(t)
