"""The autotuner's host side (no GPU): its grids, the configurations it
builds, and that it returns the fastest row of what it timed (timing stubbed
out)."""
import pytest

from paper_2208_13707_amd import mpixs as M
from paper_2208_13707_amd import tune


def test_grids_cover_every_combination():
    s = tune.schedules()
    assert len(s) == len(tune.TILES) * len(tune.MAX_WG) * len(tune.ORDERING) == len(set(s))
    assert all(t in (256, 512, 1024, 2048, 4096) for t, _, _, _ in s)
    p = tune.plain_schedules()
    assert len(p) == len(tune.FUSE) * len(tune.EAGER) == len(set(p))
    assert (-1, -1) in p                 # both thresholds off is a candidate


def test_configs_carry_the_schedule_and_keep_the_base():
    base = M.Config()
    base.timeout_ms = 1234
    base.trace_events = 64
    c = tune.config_for(1024, 4096, 1, base=base, nontemporal=2, sync=0)
    assert (c.batch_tile, c.batch_max_wg, c.batch_graph, c.batch_nontemporal, c.batch_sync) == \
        (1024, 4096, 1, 2, 0)
    assert c.timeout_ms == 1234 and c.trace_events == 64
    c = tune.plain_config(-1, 4096, base=base)
    assert (c.fuse_max_bytes, c.eager_max_bytes, c.timeout_ms) == (-1, 4096, 1234)
    assert base.fuse_max_bytes == 0 and base.eager_max_bytes == 0   # base untouched


def test_tuners_return_the_fastest_row(monkeypatch):
    times = {(256, 4096, 0, 0): 3.0, (1024, 16384, 1, 0): 1.0, (256, 32768, 0, 1): 2.0}
    monkeypatch.setattr(tune, "time_schedule",
                        lambda n, cfg, i, s, runs, warm, mr: times[(cfg.batch_tile, cfg.batch_max_wg,
                                                                    cfg.batch_graph, cfg.batch_sync)])
    best, rows = tune.tune_batch(4, None, None, candidates=list(times))
    assert len(rows) == 3 and (best["tile"], best["max_wg"], best["graph"], best["sync"]) == \
        (1024, 16384, 1, 0)
    assert best["ms_per_run"] == pytest.approx(1000.0)
    ptimes = {(-1, -1): 5e-5, (65536, 65536): 2e-5, (16384, 4096): 4e-5}
    monkeypatch.setattr(tune, "time_plain",
                        lambda n, cfg, ops, steps, warm, mr: ptimes[(cfg.fuse_max_bytes,
                                                                     cfg.eager_max_bytes)])
    best, rows = tune.tune_plain(4, None, candidates=list(ptimes))
    assert len(rows) == 3 and (best["fuse"], best["eager"]) == (65536, 65536)
    assert best["ms_per_step"] == pytest.approx(0.02)
