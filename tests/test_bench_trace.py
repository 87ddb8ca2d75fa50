"""The persistent-batch trace breakdown of bench.py on a synthetic event
ring (host logic only): each run's period, the other ranks' turn, the
launching rank's wait, the kernel, and the other ranks' completion and next
arrival, taken from POST / MATCH / DONE / COMPLETE events grouped by run."""
import types

import pytest

import bench


def _fake(events):
    M = types.SimpleNamespace(TRACE_POST=1, TRACE_MATCH=2, TRACE_DONE=3, TRACE_COMPLETE=4,
                              errname=lambda rc: str(rc))
    evs = [types.SimpleNamespace(kind=k, counter=c, value=v, time_ns=int(t * 1000), stream=s)
           for (k, c, v, t, s) in events]
    M.mpixs_world_trace = lambda world, cap: (0, len(evs), evs[-cap:])
    return M


def _run(v, posts, matches, done, completes, arrive=(64, 128), done_word=192):
    ev = [(1, arrive[i], v, t, 1 + i) for i, t in enumerate(posts)]
    ev += [(2, arrive[i], v, t, 0) for i, t in enumerate(matches)]
    ev.append((3, done_word, v, done, 0))
    ev += [(4, done_word, v, t, 1 + i) for i, t in enumerate(completes)]
    return ev


def test_batch_trace_breakdown_splits_each_run():
    ev = (_run(1, [0, 10], [15, 16], 200, [210, 220]) +
          _run(2, [230, 245], [250, 252], 400, [405, 415]) +
          _run(3, [420, 430], [440, 441], 600, [610, 611]))
    out = bench.batch_trace_breakdown(_fake(ev), None, 1000)
    assert out["runs"] == 2 and out["events"] == len(ev)
    # run 2: period 200, others' turn 245 - 200, launch wait 252 - 245,
    # kernel 400 - 252; run 3: 200, 30, 11, 159
    assert out["period_us"]["p50"] == pytest.approx(200)
    assert out["others_turn_us"]["p50"] == pytest.approx((45 + 30) / 2)
    assert out["launch_wait_us"]["p50"] == pytest.approx((7 + 11) / 2)
    assert out["kernel_us"]["p50"] == pytest.approx((148 + 159) / 2)
    # completions of runs 1 and 2: 10, 20, 5, 15; next arrivals: 20, 25, 15, 15
    assert out["done_to_complete_us"]["p50"] == pytest.approx(12.5)
    assert out["complete_to_next_post_us"]["p50"] == pytest.approx(17.5)


def test_batch_trace_breakdown_skips_runs_without_a_predecessor():
    ev = _run(5, [0, 1], [2, 3], 10, [11, 12]) + _run(7, [20, 21], [22, 23], 30, [31, 32])
    out = bench.batch_trace_breakdown(_fake(ev), None, 1000)
    assert out["runs"] == 0 and out["period_us"]["p50"] is None
