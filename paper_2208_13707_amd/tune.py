"""Schedule autotuner for persistent batches and the plain enqueue path.

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

The plain path (one enqueue call per message) has two size thresholds worth
the same treatment: up to which size a message's wait and copy run as one
kernel of at most 32 workgroups instead of a wait, a full-grid copy and a
signal (fuse_max_bytes), and up to which size a blocking send that arrives
before its receive is packed into device staging and completes on its own
stream instead of waiting for the receive (eager_max_bytes).  tune_plain
times the caller's program under each pair.
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


# plain path: (fuse_max_bytes, eager_max_bytes); -1 turns either off
FUSE = (-1, 16384, 65536, 262144, 1048576)
EAGER = (-1, 4096, 65536)


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


def plain_schedules(fuse: Sequence[int] = FUSE,
                    eager: Sequence[int] = EAGER) -> List[Tuple[int, int]]:
    return list(itertools.product(fuse, eager))


def plain_config(fuse: int, eager: int, base: M.Config = None) -> M.Config:
    c = M.Config()
    if base is not None:
        ctypes_copy(base, c)
    c.fuse_max_bytes = fuse
    c.eager_max_bytes = eager
    return c


def time_plain(nranks: int, cfg: M.Config, step_ops: Callable[[int], list], steps: int,
               warm: int, max_reqs: int, repeats: int = 3) -> float:
    """Seconds per step of the caller's plain-path program under ``cfg``:
    ``step_ops(k)`` gives each thread's driver ops for k steps; the median of
    ``repeats`` timings of ``steps`` steps after ``warm`` untimed ones."""
    sess = D.Session(nranks, cfg)
    try:
        rc, res, _ = sess.run(step_ops(warm), max_reqs=max_reqs)
        if rc:
            raise RuntimeError(f"tuning run failed: {M.errname(rc)} at thread "
                               f"{res.error_thread} op {res.error_op}")
        times = []
        for _ in range(repeats):
            rc, res, _ = sess.run(step_ops(steps), max_reqs=max_reqs)
            if rc:
                raise RuntimeError(f"tuning run failed: {M.errname(rc)}")
            times.append(res.seconds / steps)
        return sorted(times)[len(times) // 2]
    finally:
        sess.close()


def tune_plain(nranks: int, step_ops: Callable[[int], list],
               candidates: Sequence[Tuple[int, int]] = None, steps: int = 20, warm: int = 3,
               max_reqs: int = 64, base: M.Config = None, log=None) -> Tuple[Dict, List[Dict]]:
    """Grid search over (fuse_max_bytes, eager_max_bytes); returns (best,
    all) as dicts with fuse, eager and ms_per_step."""
    out = []
    for fuse, eager in (candidates or plain_schedules()):
        sec = time_plain(nranks, plain_config(fuse, eager, base), step_ops, steps, warm, max_reqs)
        row = dict(fuse=fuse, eager=eager, ms_per_step=1000.0 * sec)
        out.append(row)
        if log:
            log(f"[tune] fuse_max_bytes {fuse:8d} eager_max_bytes {eager:6d}: "
                f"{row['ms_per_step']:.4f} ms per step")
    best = min(out, key=lambda r: r["ms_per_step"])
    return best, out
