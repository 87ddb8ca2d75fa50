"""Schedule autotuner for persistent batches.

A persistent batch is planned once (descriptors, tile schedule) and then
started every step, so the schedule is worth choosing by measurement: this
module runs a grid search over the batch kernel's tile size (units per
tile), its workgroup cap and how a run is ordered across the ranks' streams
(kernels launched one by one, the launching rank's part replayed as a HIP
graph, or HIP events instead of the arrival / wait / signal kernels), timing
real runs of the caller's batch through the native driver, and returns the
fastest schedule.  It only chooses configuration values of the library
(mpixs_config.batch_tile, batch_max_wg, batch_graph, batch_sync); every run
goes through the C ABI.
"""
from __future__ import annotations

import itertools
from typing import Callable, Dict, List, Sequence, Tuple

from . import driver as D
from . import mpixs as M

TILES = (256, 1024, 4096)
MAX_WG = (4096, 16384, 32768, 65536)
# (batch_graph, batch_sync): kernels one by one, graph replay, HIP events
ORDERING = ((0, 0), (1, 0), (0, 1))


def schedules(tiles: Sequence[int] = TILES, max_wg: Sequence[int] = MAX_WG,
              ordering: Sequence[Tuple[int, int]] = ORDERING) -> List[Tuple[int, int, int, int]]:
    return [(t, m, g, s) for t, m, (g, s) in itertools.product(tiles, max_wg, ordering)]


def config_for(tile: int, max_wg: int, graph: int, base: M.Config = None,
               nontemporal: int = 0, sync: int = 0) -> M.Config:
    c = M.Config()
    if base is not None:
        ctypes_copy(base, c)
    c.batch_tile = tile
    c.batch_max_wg = max_wg
    c.batch_graph = graph
    c.batch_nontemporal = nontemporal
    c.batch_sync = sync
    return c


def ctypes_copy(src: M.Config, dst: M.Config) -> None:
    for name, _ in M.Config._fields_:
        setattr(dst, name, getattr(src, name))


def time_schedule(nranks: int, cfg: M.Config, init_ops: Callable[[], list],
                  start_ops: Callable[[int], list], runs: int, warm: int,
                  max_reqs: int, repeats: int = 3) -> float:
    """Seconds per run of the batch under ``cfg`` (init and warm-up excluded):
    the median of ``repeats`` timings of ``runs`` back-to-back runs."""
    sess = D.Session(nranks, cfg)
    try:
        for ops in (init_ops(), start_ops(warm)):
            rc, res, _ = sess.run(ops, max_reqs=max_reqs)
            if rc:
                raise RuntimeError(f"tuning run failed: {M.errname(rc)} at thread "
                                   f"{res.error_thread} op {res.error_op}")
        times = []
        for _ in range(repeats):
            rc, res, _ = sess.run(start_ops(runs), max_reqs=max_reqs)
            if rc:
                raise RuntimeError(f"tuning run failed: {M.errname(rc)}")
            times.append(res.seconds / runs)
        return sorted(times)[len(times) // 2]
    finally:
        sess.close()


def tune_batch(nranks: int, init_ops: Callable[[], list], start_ops: Callable[[int], list],
               candidates: Sequence[Tuple[int, int, int, int]] = None, runs: int = 10,
               warm: int = 2, max_reqs: int = 64, log=None) -> Tuple[Dict, List[Dict]]:
    """Grid search; returns (best, all) as dicts with tile, max_wg, graph,
    sync and ms_per_run.  ``init_ops()`` gives each thread's driver ops that record
    the group and end it with GROUP_INIT into batch slot 0;
    ``start_ops(k)`` gives k BATCH_START ops per thread."""
    out = []
    for tile, max_wg, graph, sync in (candidates or schedules()):
        sec = time_schedule(nranks, config_for(tile, max_wg, graph, sync=sync), init_ops,
                            start_ops, runs, warm, max_reqs)
        row = dict(tile=tile, max_wg=max_wg, graph=graph, sync=sync, ms_per_run=1000.0 * sec)
        out.append(row)
        if log:
            log(f"[tune] tile {tile:5d} max_wg {max_wg:6d} graph {graph} sync {sync}: "
                f"{row['ms_per_run']:.3f} ms per run")
    best = min(out, key=lambda r: r["ms_per_run"])
    return best, out
