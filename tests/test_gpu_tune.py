"""The autotuner on the GPU, through the C ABI: it times real runs of the
caller's program under each candidate configuration and returns the fastest,
and the program's results under the chosen configuration are exact.
A persistent ring batch (4 ranks, a contiguous and a vector message per
rank) over three batch schedules, and a blocking ring (4 ranks, 8 KiB
messages, so eager sends apply) over three (fuse, eager) threshold pairs."""
import sys

import pytest

pytestmark = pytest.mark.gpu

N = 4


def _say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def _bufs():
    import torch
    src = [torch.arange(8192, dtype=torch.int32, device="cuda") * (r + 1) for r in range(N)]
    dst = [torch.zeros(8192, dtype=torch.int32, device="cuda") for _ in range(N)]
    torch.cuda.synchronize()
    return src, dst


def _vector(M):
    rc, t = M.mpixs_type_vector(512, 3, 8, M.FLOAT32)
    assert rc == 0
    rc, t = M.mpixs_type_commit(t)
    assert rc == 0
    return t


def test_tune_batch_picks_the_fastest_schedule_and_runs_it_exactly():
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    from paper_2208_13707_amd import tune
    _say("tune_batch: 4-rank persistent ring, three schedules")
    src, dst = _bufs()
    vt = _vector(M)

    def init_ops():
        out = []
        for r in range(N):
            right, left = (r + 1) % N, (r - 1) % N
            s, d = src[r].data_ptr(), dst[r].data_ptr()
            out.append(D.ops_array([
                dict(kind=D.GROUP_START),
                dict(kind=D.ISEND, peer=right, tag=1, count=1024, datatype=M.INT32, buf=s, req=0),
                dict(kind=D.ISEND, peer=right, tag=2, count=1, datatype=vt, buf=s + 4096, req=1),
                dict(kind=D.IRECV, peer=left, tag=1, count=1024, datatype=M.INT32, buf=d, req=2),
                dict(kind=D.IRECV, peer=left, tag=2, count=1, datatype=vt, buf=d + 4096, req=3),
                dict(kind=D.WAITALL, req=0, nreq=4),
                dict(kind=D.GROUP_INIT, req=0)]))
        return out

    def start_ops(k):
        return [D.ops_array([dict(kind=D.BATCH_START, req=0)] * k) for _ in range(N)]

    cands = [(256, 4096, 0, 0), (1024, 16384, 1, 0), (256, 32768, 0, 1)]
    best, rows = tune.tune_batch(N, init_ops, start_ops, candidates=cands, runs=5, warm=1,
                                 max_reqs=5)
    assert len(rows) == 3 and all(r["ms_per_run"] > 0 for r in rows)
    assert best["ms_per_run"] == min(r["ms_per_run"] for r in rows)
    sess = D.Session(N, tune.config_for(best["tile"], best["max_wg"], best["graph"],
                                        sync=best["sync"]))
    try:
        for x in dst:
            x.zero_()
        torch.cuda.synchronize()
        for ops in (init_ops(), start_ops(2)):
            rc, _, _ = sess.run(ops, max_reqs=5)
            assert rc == 0, M.errname(rc)
        for r in range(N):
            want = src[(r - 1) % N].cpu()
            got = dst[r].cpu()
            assert torch.equal(got[:1024], want[:1024]), r
            # the vector: 512 blocks of 3 floats at a stride of 8, from byte 4096
            w = want[1024:1024 + 512 * 8].view(512, 8)[:, :3]
            g = got[1024:1024 + 512 * 8].view(512, 8)
            assert torch.equal(g[:, :3], w) and not g[:, 3:].any(), r
    finally:
        torch.cuda.synchronize()
        sess.close()
        M.mpixs_type_free(vt)


def test_tune_plain_picks_the_fastest_thresholds_and_runs_them_exactly():
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    from paper_2208_13707_amd import tune
    _say("tune_plain: 4-rank blocking ring of 8 KiB messages, three threshold pairs")
    src, dst = _bufs()

    def step_ops(k):
        out = []
        for r in range(N):
            right, left = (r + 1) % N, (r - 1) % N
            rows = []
            for s in range(k):
                snd = dict(kind=D.SEND, peer=right, tag=s, count=2048, datatype=M.INT32,
                           buf=src[r].data_ptr())
                rcv = dict(kind=D.RECV, peer=left, tag=s, count=2048, datatype=M.INT32,
                           buf=dst[r].data_ptr())
                rows += [snd, rcv] if r % 2 == 0 else [rcv, snd]
            out.append(D.ops_array(rows))
        return out

    cands = [(-1, -1), (65536, 65536), (16384, 4096)]
    best, rows = tune.tune_plain(N, step_ops, candidates=cands, steps=10, warm=2, max_reqs=2)
    assert len(rows) == 3 and all(r["ms_per_step"] > 0 for r in rows)
    assert best["ms_per_step"] == min(r["ms_per_step"] for r in rows)
    sess = D.Session(N, tune.plain_config(best["fuse"], best["eager"]))
    try:
        for x in dst:
            x.zero_()
        torch.cuda.synchronize()
        rc, _, _ = sess.run(step_ops(3), max_reqs=2)
        assert rc == 0, M.errname(rc)
        for r in range(N):
            assert torch.equal(dst[r][:2048], src[(r - 1) % N][:2048]), r
            assert not dst[r][2048:].any(), r
    finally:
        torch.cuda.synchronize()
        sess.close()
