"""Serving harness on the GPU: every request's result equals its expected
value, alone and in the mix (requests admitted as memory frees up), and
the host-synchronised comparison path gives the same results.

The expected values come from the payload definition (SplitMix64 bytes) and
the oracle's fold, computed on the host.  An allreduce request's checksum
covers every rank's output (rank r weighted by 2r + 1), so with all outputs
equal to the fold it is n^2 times the fold's checksum.  At the serving
configuration's shape (64 ranks, requests of 64 B to 4 MiB) the bytes of a
sample of requests -- every rank's output for the sampled allreduces -- are
also captured on the device before their checksum and compared in full.
"""
import sys

import numpy as np
import pytest

from oracle import reduce as red
from workloads import configs as C
from workloads import payload

pytestmark = pytest.mark.gpu

M64 = (1 << 64) - 1


def checksum(b: np.ndarray) -> int:
    j = np.arange(1, b.size + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return int((b.astype(np.uint64) * j).sum(dtype=np.uint64))


def fold_bytes(q, nranks):
    ins = [payload.fill(q["seed"] + r, q["bytes"]).view(np.int32) for r in range(nranks)]
    return red.fold("sum", ins).view(np.uint8)


def expected(q, nranks):
    if q["kind"] == 2:
        return (nranks * nranks * checksum(fold_bytes(q, nranks))) & M64
    return checksum(payload.fill(q["seed"], q["bytes"]))


def test_serving_results_alone_and_in_mix():
    from paper_2208_13707_amd import driver as D
    n = 8
    sched = C.serving_schedule(rate=3e5, nreq=240, nranks=n, max_bytes=1 << 17, seed=3)
    print(f"[gpu-case] serving {len(sched)} requests, 8 ranks", file=sys.stderr, flush=True)
    sess = D.Session(n)
    try:
        # a 4 MiB budget: later requests wait for earlier ones to free memory
        rc, res, wall = sess.serve(sched, budget_bytes=4 << 20)
        assert rc == 0
        assert np.all(res["error"] == 0)
        assert np.all(res["done_us"] >= res["admit_us"])
        want = [expected(q, n) for q in sched]
        assert [int(x) for x in res["checksum"]] == want
        sample = [i for i, q in enumerate(sched) if q["kind"] == 2][:3] + [0, 1, 5, 17, 101]
        for i in sample:
            q = dict(sched[i])
            q["arrival_us"] = 0.0
            rc, r1, _ = sess.serve([q], budget_bytes=4 << 20)
            assert rc == 0 and int(r1["checksum"][0]) == want[i]
    finally:
        sess.close()


def test_serving_host_synced_path_gives_identical_results():
    """The comparison path (host-synchronised calls, §2.4) on the same
    schedule: every checksum equals the enqueue path's and the expected one."""
    from paper_2208_13707_amd import driver as D
    n = 16
    sched = C.serving_schedule(rate=1e5, nreq=200, nranks=n, max_bytes=1 << 18, seed=5)
    print(f"[gpu-case] serving {len(sched)} requests, 16 ranks, enqueue and host-synced",
          file=sys.stderr, flush=True)
    sess = D.Session(n)
    try:
        want = [expected(q, n) for q in sched]
        got = {}
        for mode in (0, D.SERVE_HOST_SYNCED):
            rc, res, wall = sess.serve(sched, budget_bytes=64 << 20, flags=mode)
            assert rc == 0, f"mode {mode}: {rc}"
            assert np.all(res["error"] == 0)
            got[mode] = [int(x) for x in res["checksum"]]
            assert got[mode] == want, f"mode {mode}"
        assert got[0] == got[D.SERVE_HOST_SYNCED]
    finally:
        sess.close()


def test_serving_64_ranks_4mib_bytes_captured():
    import torch
    from paper_2208_13707_amd import driver as D
    n = 64
    budget = 512 << 20     # the largest allreduce (2 x 64 x 4 MiB) just fits: admissions wait
    sched = C.serving_schedule(rate=3e4, nreq=320, nranks=n, max_bytes=4 << 20, seed=11)
    big_ar = [i for i, q in enumerate(sched) if q["kind"] == 2]
    assert max(2 * n * ((sched[i]["bytes"] + 255) // 256 * 256) for i in big_ar) <= budget
    p2p = sorted((i for i, q in enumerate(sched) if q["kind"] != 2),
                 key=lambda i: -sched[i]["bytes"])
    # captured in full: the three largest allreduces, the six largest
    # point-to-point requests and four small ones
    sample = sorted(big_ar, key=lambda i: -sched[i]["bytes"])[:3] + p2p[:6] + p2p[-4:]
    offs, at = [], 0
    for i in sample:
        offs.append(at)
        at += sched[i]["bytes"] * (n if sched[i]["kind"] == 2 else 1)
        at = (at + 255) // 256 * 256
    cap = torch.full((at,), 0xA5, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    print(f"[gpu-case] serving {len(sched)} requests, 64 ranks, <= 4 MiB, 512 MiB budget, "
          f"{len(sample)} captured ({at >> 20} MiB)", file=sys.stderr, flush=True)
    sess = D.Session(n)
    try:
        rc, res, wall = sess.serve(sched, budget_bytes=budget,
                                   capture=list(zip(sample, offs)), capture_dev=cap.data_ptr())
        assert rc == 0
        assert np.all(res["error"] == 0)
        assert np.all(res["done_us"] >= res["admit_us"])
        got = cap.cpu().numpy()
        for i, o in zip(sample, offs):
            q = sched[i]
            if q["kind"] == 2:
                want = fold_bytes(q, n)
                b = q["bytes"]
                for r in range(n):
                    seg = got[o + r * b: o + (r + 1) * b]
                    assert np.array_equal(seg, want), f"request {i} (allreduce) rank {r}"
            else:
                want = payload.fill(q["seed"], q["bytes"])
                assert np.array_equal(got[o: o + q["bytes"]], want), f"request {i}"
        want = [expected(q, n) for q in sched]
        bad = [i for i, q in enumerate(sched) if int(res["checksum"][i]) != want[i]]
        assert not bad, f"checksums differ for requests {bad[:10]}"
    finally:
        sess.close()
