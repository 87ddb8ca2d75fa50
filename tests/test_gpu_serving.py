"""Serving harness on the GPU: every request's result equals its expected
value, alone and in the mix (requests admitted as memory frees up)."""
import sys

import numpy as np
import pytest

from oracle import reduce as red
from workloads import configs as C
from workloads import payload

pytestmark = pytest.mark.gpu


def checksum(b: np.ndarray) -> int:
    j = np.arange(1, b.size + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return int((b.astype(np.uint64) * j).sum(dtype=np.uint64))


def expected(q, nranks):
    if q["kind"] == 2:
        ins = [payload.fill(q["seed"] + r, q["bytes"]).view(np.int32) for r in range(nranks)]
        return checksum(red.fold("sum", ins).view(np.uint8))
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
