#!/usr/bin/env python3
"""Benchmark of stream-ordered enqueue traffic on one MI355X.

Default workload (a "step" = one pass of the whole batch): 10,000 enqueued
send/recv pairs among 32 ranks (host threads, one HIP stream each), sizes
log-uniform from 8 B to 256 KiB, tags 0..63, 30 % vector datatypes, the
rest contiguous; every rank isends all its messages, irecvs all its
messages and waits for all of them.  The same batch runs four ways: a
persistent batch (planned once, one batch kernel per step; the headline), a
one-shot group per step, the plain enqueue path (one copy per message) and
the host-synchronised path; all four must give identical bytes, and the
oracle checks one batch.

Prints ONE JSON line: messages/s (value), algorithmic GB/s and HBM fraction,
the host-synchronised rate and speedups, p50/p99 batch latency, the roofline
of the dominant kernel (the batch kernel), the CPU oracle timed on one
batch, and two more configurations: the 16-rank allreduce at 64 MiB per rank
(float32 and int64: calls/s, HBM fraction, host-synchronised calls/s) and the
8-rank ring halo of vector(43690, 3, 8) float32 messages with tag = step
(value: the plain enqueue path; grouped, persistent and host-synchronised
beside it).

Other workloads (--workload): halo, pingpong (2 ranks, 1000 x 4 KiB int32),
allreduce (16 ranks, SUM, --bytes per rank, --dtype), copy (one contiguous
message of --bytes between two ranks), serve, nto1, and hostrate (CPU only:
the host message-rate model of three engine locking policies).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published


def measured_traffic(key, workgroups=None):
    """HBM bytes per launch of a kernel from the committed counter runs, or
    None when the device sources that kernel is built from changed since
    those counters were taken, or when the counters were taken at another
    grid size than the launch being reported (`workgroups`)."""
    import hashlib
    import json as _json
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        rec = _json.load(open(path))
    except OSError:
        return None
    ent = rec.get(key)
    if not ent:
        return None
    src = os.path.join(ROOT, "paper_2208_13707_amd", "csrc")
    h = hashlib.sha256()
    for name in ent["sources"]:
        with open(os.path.join(src, name), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != ent.get("sources_sha256"):
        return None
    if workgroups is not None and ent.get("workgroups") != workgroups:
        return None
    return ent["read_bytes"] + ent["write_bytes"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if len(xs) else None


# ------------------------------------------------------------------ helpers
def make_vector(M, count, bl, stride, base):
    rc, t = M.mpixs_type_vector(count, bl, stride, base)
    assert rc == 0
    rc, t = M.mpixs_type_commit(t)
    assert rc == 0
    return t


def halo_ops(D, r, n, A, H, vt, steps, tag0, mode, marks=False, status_ptr=0, grouped=False):
    right, left = (r + 1) % n, (r - 1) % n
    rows = []
    a0, a3 = A.data_ptr(), A.data_ptr() + 12
    h0, h3 = H.data_ptr(), H.data_ptr() + 12
    for s in range(steps):
        tag = tag0 + s
        if marks:
            rows.append(dict(kind=D.MARK, req=2 * s))
        if grouped:
            rows.append(dict(kind=D.GROUP_START))
        if mode == 0:
            rows += [dict(kind=D.ISEND, peer=right, tag=tag, count=1, datatype=vt, buf=a0, req=0),
                     dict(kind=D.ISEND, peer=left, tag=tag, count=1, datatype=vt, buf=a3, req=1),
                     dict(kind=D.RECV, peer=left, tag=tag, count=1, datatype=vt, buf=h0,
                          status=status_ptr),
                     dict(kind=D.RECV, peer=right, tag=tag, count=1, datatype=vt, buf=h3),
                     dict(kind=D.WAITALL, req=0, nreq=2)]
        else:
            # blocking, deadlock-free ring order for an even number of ranks
            sr = dict(kind=D.SEND, peer=right, tag=tag, count=1, datatype=vt, buf=a0)
            rl = dict(kind=D.RECV, peer=left, tag=tag, count=1, datatype=vt, buf=h0,
                      status=status_ptr)
            sl = dict(kind=D.SEND, peer=left, tag=tag, count=1, datatype=vt, buf=a3)
            rr = dict(kind=D.RECV, peer=right, tag=tag, count=1, datatype=vt, buf=h3)
            rows += [sr, rl, sl, rr] if r % 2 == 0 else [rl, sr, rr, sl]
        if grouped:
            rows.append(dict(kind=D.GROUP_END))
        if marks:
            rows.append(dict(kind=D.MARK, req=2 * s + 1))
    return D.ops_array(rows)


def halo_persistent_ops(D, r, n, A, H, vt, steps, init=False, marks=False):
    """init: record one halo step (tag 0) as persistent batch slot 0;
    else: start it ``steps`` times."""
    if init:
        right, left = (r + 1) % n, (r - 1) % n
        a0, a3 = A.data_ptr(), A.data_ptr() + 12
        h0, h3 = H.data_ptr(), H.data_ptr() + 12
        rows = [dict(kind=D.GROUP_START),
                dict(kind=D.ISEND, peer=right, tag=0, count=1, datatype=vt, buf=a0, req=0),
                dict(kind=D.ISEND, peer=left, tag=0, count=1, datatype=vt, buf=a3, req=1),
                dict(kind=D.RECV, peer=left, tag=0, count=1, datatype=vt, buf=h0),
                dict(kind=D.RECV, peer=right, tag=0, count=1, datatype=vt, buf=h3),
                dict(kind=D.WAITALL, req=0, nreq=2),
                dict(kind=D.GROUP_INIT, req=0)]
        return D.ops_array(rows)
    rows = []
    for s in range(steps):
        if marks:
            rows.append(dict(kind=D.MARK, req=2 * s))
        rows.append(dict(kind=D.BATCH_START, req=0))
        if marks:
            rows.append(dict(kind=D.MARK, req=2 * s + 1))
    return D.ops_array(rows)


def batch_nt_used(flag, payload):
    """Whether the batch kernel uses nontemporal accesses (the library's rule
    for mpixs_config.batch_nontemporal)."""
    return flag == 1 or (flag == 0 and payload >= 64 << 20)


def halo_batch_cfg(M, args):
    """World configuration of the persistent halo (batch schedule flags)."""
    c = M.Config()
    c.batch_tile = args.batch_tile
    c.batch_max_wg = args.batch_max_wg
    c.batch_graph = args.batch_graph
    c.batch_nontemporal = args.batch_nt
    c.batch_sync = args.batch_sync
    return c


def time_batch_kernel(sess, reps):
    """Average duration of a persistent batch's kernel (slot 0 of rank 0's
    handles), launched back to back between one pair of HIP events."""
    import ctypes
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    f = M.lib().mpixs_debug_time_batch
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)]
    f.restype = ctypes.c_int
    hs = D.hip_stream_create()
    avg, nbytes, nwg = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int()
    rc = f(sess.batches[0][0], hs, reps, ctypes.byref(avg), ctypes.byref(nbytes), ctypes.byref(nwg))
    D.hip_stream_destroy(hs)
    if rc:
        raise RuntimeError(f"mpixs_debug_time_batch: {M.errname(rc)}")
    return avg.value, nbytes.value, nwg.value


def close_checked(sess):
    """Close a session after checking that no rank's stream recorded an
    asynchronous error (a copy or wait that failed on the device)."""
    errs = sess.stream_errors()
    sess.close()
    if any(errs):
        raise RuntimeError(f"asynchronous stream errors: {errs}")


def run_checked(sess, ops, mode=0, nmarks=0, max_reqs=64, enqueue=False):
    """Runs the rank programs; returns (seconds, marks), or with enqueue=True
    (seconds, marks, enqueue_seconds): when the last rank thread returned
    from its last call, before the stream syncs (the host's share)."""
    from paper_2208_13707_amd import mpixs as M
    rc, res, marks = sess.run(ops, mode=mode, nmarks=nmarks, max_reqs=max_reqs)
    if rc:
        raise RuntimeError(f"driver: {M.errname(rc)} at thread {res.error_thread} op {res.error_op}")
    # every rank thread of the runner has synchronised its own stream: the
    # results may be read on torch's stream now, with no device-wide sync
    if enqueue:
        return res.seconds, marks, res.enqueue_seconds
    return res.seconds, marks


def step_latencies(marks, steps):
    lat = []
    for s in range(steps):
        start = marks[:, 2 * s].min()
        end = marks[:, 2 * s + 1].max()
        lat.append((end - start) * 1000.0)   # us
    return lat


# ------------------------------------------------------------------ halo
def vector_copy_roofline(count, k):
    """The halo's dominant kernel at its real shape: the typemap copy of one
    vector(count, 3, 8, float32) message into the same vector type.  Its data
    kernel is launched k times back to back on one stream between one pair
    of HIP events (on that stream), so the average is a per-launch duration
    that a short kernel's per-launch event pairs would bury in marker
    overhead."""
    import ctypes
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    from workloads import configs as C
    p = C.ring_halo(count=count, steps=1, nranks=2)
    A = torch.from_numpy(p.buffers[0]["A"].copy()).cuda()
    H = torch.from_numpy(p.buffers[1]["H"].copy()).cuda()
    torch.cuda.synchronize()
    vt = make_vector(M, count, 3, 8, M.FLOAT32)
    f = M.lib().mpixs_debug_time_copy
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int32, ctypes.c_void_p,
                  ctypes.c_int, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                  ctypes.POINTER(ctypes.c_int)]
    f.restype = ctypes.c_int
    hs = D.hip_stream_create()
    avg = ctypes.c_double()
    w = ctypes.c_int()
    rc = f(hs, A.data_ptr(), 1, vt, H.data_ptr(), 1, vt, k, ctypes.byref(avg), ctypes.byref(w))
    D.hip_stream_destroy(hs)
    if rc:
        raise RuntimeError(f"mpixs_debug_time_copy: {M.errname(rc)}")
    per_launch = 2 * 12 * count
    ach = per_launch / (avg.value * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS,
            "traffic": measured_traffic(f"halo_vector_copy_count{count}"),
            "kernel": f"mpixs::k_copy<{w.value}, 1, 1, false>", "bytes_per_launch": per_launch,
            "avg_launch_us": avg.value, "launches_timed": k,
            "note": "data kernel of one halo message, launched back to back between one event pair"}


def pattern_rates(payload=128 << 20, reps=20, bls=tuple(range(1, 17)), log_rows=False):
    """The copy kernel of the library on one message of `payload` bytes in
    each layout pattern (launched back to back between one pair of HIP
    events on its stream): contiguous, and vector(c, bl, 2 bl, float32) on
    both sides (half of every extent used) for each block length bl, as
    algorithmic TB/s (2 x payload / time).  These are what the memory system
    allows for each pattern: below 64-byte blocks a vector destination is
    written in partial 64-byte granules and its source read in whole lines."""
    import ctypes
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    f = M.lib().mpixs_debug_time_copy
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int32, ctypes.c_void_p,
                  ctypes.c_int, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                  ctypes.POINTER(ctypes.c_int)]
    f.restype = ctypes.c_int
    src = torch.empty(2 * payload, dtype=torch.uint8, device="cuda").fill_(7)
    dst = torch.zeros(2 * payload, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    hs = D.hip_stream_create()
    out = {}
    try:
        cases = [("contig", None)] + [(bl, bl) for bl in bls]
        for key, bl in cases:
            if bl is None:
                st = rt = M.UINT8
                cnt = payload
            else:
                st = rt = make_vector(M, payload // (4 * bl), bl, 2 * bl, M.FLOAT32)
                cnt = 1
            avg = ctypes.c_double()
            w = ctypes.c_int()
            rc = f(hs, src.data_ptr(), cnt, st, dst.data_ptr(), cnt, rt, reps, ctypes.byref(avg),
                   ctypes.byref(w))
            if bl is not None:
                M.mpixs_type_free(st)
            if rc:
                raise RuntimeError(f"mpixs_debug_time_copy: {M.errname(rc)}")
            pay = payload if bl is None else payload // (4 * bl) * 4 * bl
            out[key] = 2 * pay / (avg.value * 1e-6) / 1e12
            if log_rows:
                log(f"[patterns] {'contiguous' if bl is None else f'vector bl={bl:2d} ({4 * bl:3d} B blocks)'}: "
                    f"{avg.value:8.1f} us, {out[key]:.2f} TB/s algorithmic")
    finally:
        D.hip_stream_destroy(hs)
        del src, dst
    return out


def pattern_bound_us(msgs, rates):
    """Lower bound on a batch kernel's time: every message at its pattern's
    copy rate (contiguous, or the vector block length's), no overheads."""
    t = 0.0
    for m in msgs:
        tree = m["tree"]
        key = tree[2] if isinstance(tree, tuple) and tree[0] == "vector" else "contig"
        t += 2 * m["size"] / (rates[key] * 1e12)
    return t * 1e6


def halo_cpu_baseline(count, budget_s=15.0):
    """The oracle as it stands on a bounded sample of the same workload."""
    from oracle import simulate as sim
    from workloads import configs as C
    t0 = time.perf_counter()
    sim.run(C.ring_halo(count=count, steps=1))
    t1 = time.perf_counter() - t0
    steps = int(max(1, min(100, budget_s / max(t1, 1e-3))))
    p = C.ring_halo(count=count, steps=steps)
    t0 = time.perf_counter()
    sim.run(p)
    dt = time.perf_counter() - t0
    msgs = 16 * steps
    return {"value": msgs / dt, "unit": "msgs/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} ring-halo steps ({msgs} messages of {12 * count} bytes), "
                      f"8 ranks, single-threaded numpy simulator, {dt:.1f} s"}


def bench_halo(args):
    import numpy as np
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    from workloads import configs as C

    n, steps, warm = 8, args.steps, args.warmup
    if args.kernel_only:
        # counter runs: plan one persistent halo step (no GPU waits) and launch
        # its batch kernel only
        p = C.ring_halo(count=args.count, steps=1)
        A = [torch.from_numpy(p.buffers[r]["A"].copy()).cuda() for r in range(n)]
        H = [torch.from_numpy(p.buffers[r]["H"].copy()).cuda() for r in range(n)]
        vt = make_vector(M, args.count, 3, 8, M.FLOAT32)
        torch.cuda.synchronize()
        sess = D.Session(n, halo_batch_cfg(M, args))
        run_checked(sess, [halo_persistent_ops(D, r, n, A[r], H[r], vt, 0, init=True)
                           for r in range(n)])
        us, payload, nwg = time_batch_kernel(sess, steps)
        close_checked(sess)
        return {"workload": "halo batch kernel only", "avg_launch_us": us,
                "payload_bytes": payload, "workgroups": nwg, "launches": steps + 1}
    counts = [args.count] + ([c for c in C.HALO_COUNTS if c != args.count] if args.sweep else [])
    out_sweep = []
    headline = None
    for count in counts:
        p = C.ring_halo(count=count, steps=1)
        A = [torch.from_numpy(p.buffers[r]["A"].copy()).cuda() for r in range(n)]
        H = [torch.from_numpy(p.buffers[r]["H"].copy()).cuda() for r in range(n)]
        torch.cuda.synchronize()
        vt = make_vector(M, count, 3, 8, M.FLOAT32)
        payload = 12 * count
        res = {"count": count, "payload_bytes": payload}
        fuse = args.fuse_max_bytes
        if args.tune_plain:
            # the plain path's fuse threshold chosen by timing this program
            # (the halo has no blocking sends, so the eager threshold is moot)
            from paper_2208_13707_amd import tune
            best, rows = tune.tune_plain(
                n, lambda k: [halo_ops(D, r, n, A[r], H[r], vt, k, 0, 0) for r in range(n)],
                candidates=[(f, 0) for f in tune.FUSE], steps=max(10, min(steps, 50)), warm=5,
                log=log)
            fuse = best["fuse"]
            res["tuned_plain"] = {"chosen": best, "grid": rows}
        # ---- enqueue path: warmup, then K timed steps
        pc = None
        if fuse is not None or args.trace:
            pc = M.Config()
            if fuse is not None:
                pc.fuse_max_bytes = fuse
            if args.trace:
                pc.trace_events = 1 << 16
        sess = D.Session(n, pc)
        ops = [halo_ops(D, r, n, A[r], H[r], vt, warm, 0, 0) for r in range(n)]
        run_checked(sess, ops)
        ops = [halo_ops(D, r, n, A[r], H[r], vt, steps, 0, 0) for r in range(n)]
        torch.cuda.synchronize()
        sec, _, enq = run_checked(sess, ops, enqueue=True)
        st = sess.stats()
        msgs = 16 * steps
        res.update(msgs_per_s=msgs / sec, ms_per_step=1000 * sec / steps,
                   enqueue_ms_per_step=1000 * enq / steps,
                   gbps_payload=msgs * payload / sec / 1e9,
                   gbps_algorithmic=2 * msgs * payload / sec / 1e9,
                   kernels_per_msg=(st.kernels_post + st.kernels_wait + st.kernels_copy) /
                   max(1, 16 * (steps + warm)))
        if args.trace:
            # the timed steps' messages, one by one on the device (the ring
            # holds the last 16,384 messages: all of the timed steps')
            res["trace"] = trace_breakdown(M, sess.world, min(1 << 16, 4 * 16 * steps))
            log(f"[halo] count={count} trace: {json.dumps(res['trace'])}")
        # ---- latency pass (HIP events at step boundaries on every stream)
        ops = [halo_ops(D, r, n, A[r], H[r], vt, steps, 0, 0, marks=True) for r in range(n)]
        _, marks = run_checked(sess, ops, nmarks=2 * steps)
        lat = step_latencies(marks, steps)
        res.update(p50_step_us=pct(lat, 50), p99_step_us=pct(lat, 99))
        close_checked(sess)
        # ---- batched: every step's operations form one group (one kernel)
        Hg = [torch.from_numpy(p.buffers[r]["H"].copy()).cuda() for r in range(n)]
        torch.cuda.synchronize()
        sess = D.Session(n)
        ops = [halo_ops(D, r, n, A[r], Hg[r], vt, warm, 20000, 0, grouped=True) for r in range(n)]
        run_checked(sess, ops)
        ops = [halo_ops(D, r, n, A[r], Hg[r], vt, steps, 20000, 0, grouped=True) for r in range(n)]
        sec_g, _ = run_checked(sess, ops)
        ops = [halo_ops(D, r, n, A[r], Hg[r], vt, steps, 20000, 0, marks=True, grouped=True)
               for r in range(n)]
        _, marks = run_checked(sess, ops, nmarks=2 * steps)
        lat_g = step_latencies(marks, steps)
        close_checked(sess)
        res.update(grouped_msgs_per_s=msgs / sec_g, grouped_ms_per_step=1000 * sec_g / steps,
                   grouped_p50_step_us=pct(lat_g, 50), grouped_p99_step_us=pct(lat_g, 99))
        for r in range(n):
            if not torch.equal(Hg[r], H[r]):
                raise AssertionError(f"rank {r}: grouped halo differs from the plain path")
        # ---- persistent: one step recorded once, started every step
        Hp = [torch.from_numpy(p.buffers[r]["H"].copy()).cuda() for r in range(n)]
        torch.cuda.synchronize()
        sess = D.Session(n, halo_batch_cfg(M, args))
        run_checked(sess, [halo_persistent_ops(D, r, n, A[r], Hp[r], vt, 0, init=True)
                           for r in range(n)])
        run_checked(sess, [halo_persistent_ops(D, r, n, A[r], Hp[r], vt, warm) for r in range(n)])
        sec_p, _ = run_checked(sess, [halo_persistent_ops(D, r, n, A[r], Hp[r], vt, steps)
                                      for r in range(n)])
        _, marks = run_checked(sess, [halo_persistent_ops(D, r, n, A[r], Hp[r], vt, steps,
                                                          marks=True) for r in range(n)],
                               nmarks=2 * steps)
        lat_p = step_latencies(marks, steps)
        if count == args.count:
            bk_us, bk_payload, bk_wg = time_batch_kernel(sess, max(20, steps))
            res["batch_kernel"] = {"avg_launch_us": bk_us, "payload_bytes": bk_payload,
                                   "workgroups": bk_wg}
        close_checked(sess)
        res.update(persistent_msgs_per_s=msgs / sec_p, persistent_ms_per_step=1000 * sec_p / steps,
                   persistent_p50_step_us=pct(lat_p, 50), persistent_p99_step_us=pct(lat_p, 99))
        for r in range(n):
            if not torch.equal(Hp[r], H[r]):
                raise AssertionError(f"rank {r}: persistent halo differs from the plain path")
        # ---- correctness against the oracle (sampled: after any step, H holds
        # the neighbours' halo columns; the oracle runs one full-size step)
        if count == args.count:
            from oracle import simulate as sim
            ref = sim.run(p)
            for r in range(n):
                got = H[r].cpu().numpy()
                if not np.array_equal(got, ref.buffers[r]["H"]):
                    raise AssertionError(f"rank {r}: halo differs from the oracle")
        # ---- host-synchronised path, same workload and buffers
        if not args.no_host_synced:
            H2 = [torch.from_numpy(p.buffers[r]["H"].copy()).cuda() for r in range(n)]
            torch.cuda.synchronize()
            hs_steps = max(1, min(steps, args.hs_steps))
            sess = D.Session(n)
            ops = [halo_ops(D, r, n, A[r], H2[r], vt, min(warm, 5), 10000, 1) for r in range(n)]
            run_checked(sess, ops, mode=1)
            ops = [halo_ops(D, r, n, A[r], H2[r], vt, hs_steps, 10000, 1) for r in range(n)]
            sec_hs, _ = run_checked(sess, ops, mode=1)
            close_checked(sess)
            res["host_synced_msgs_per_s"] = 16 * hs_steps / sec_hs
            res["speedup_vs_host_synced"] = res["msgs_per_s"] / res["host_synced_msgs_per_s"]
            for r in range(n):
                if not torch.equal(H2[r], H[r]):
                    raise AssertionError(f"rank {r}: host-synced path differs from enqueue path")
        if count == args.count:
            headline = res
        out_sweep.append(res)
        log(f"[halo] count={count}: {res['msgs_per_s']:.0f} msgs/s "
            f"(enqueue {1000 * res['enqueue_ms_per_step']:.1f} of {1000 * res['ms_per_step']:.1f} us/step), "
            f"grouped {res['grouped_msgs_per_s']:.0f} msgs/s, "
            f"persistent {res['persistent_msgs_per_s']:.0f} msgs/s, "
            f"{res['gbps_algorithmic']:.1f} GB/s alg, "
            f"host-synced {res.get('host_synced_msgs_per_s', 0):.0f} msgs/s")

    h = headline
    variants = {"plain": ("msgs_per_s", "ms_per_step", "p50_step_us", "p99_step_us",
                          "plain enqueue (one copy per message)"),
                "grouped": ("grouped_msgs_per_s", "grouped_ms_per_step", "grouped_p50_step_us",
                            "grouped_p99_step_us", "grouped (each step one group)"),
                "persistent": ("persistent_msgs_per_s", "persistent_ms_per_step",
                               "persistent_p50_step_us", "persistent_p99_step_us",
                               "persistent batch (one step recorded once, started every step)")}
    best = max(variants, key=lambda v: h[variants[v][0]])
    kv, km, k50, k99, vname = variants[best]
    value, ms_step = h[kv], h[km]
    if best in ("persistent", "grouped") and "batch_kernel" in h:
        # both variants run one batch kernel per step (a one-shot group reads
        # its descriptors from host-pinned memory, a persistent one from
        # device memory); it is timed on the persistent plan
        bk = h["batch_kernel"]
        per_launch = 2 * bk["payload_bytes"]
        ach = per_launch / (bk["avg_launch_us"] * 1e-6) / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS,
                "traffic": measured_traffic(f"halo_batch_count{h['count']}", bk["workgroups"]),
                "kernel": f"mpixs::k_batch<{args.batch_tile}, "
                          f"{'true' if batch_nt_used(args.batch_nt, bk['payload_bytes']) else 'false'}>",
                "bytes_per_launch": per_launch,
                "avg_launch_us": bk["avg_launch_us"], "launches_timed": max(20, steps),
                "workgroups": bk["workgroups"],
                "note": "batch kernel of one halo step (16 messages), launched back to back "
                        "between one event pair"}
    else:
        roof = vector_copy_roofline(h["count"], steps)
    # the achievable copy peak of this GPU, measured in the same run
    cp = achievable_copy_gbps()
    roof["achievable_copy_GBps"] = cp
    roof["frac_of_achievable"] = roof["achieved"] / cp
    log(f"[halo] 1 GiB copy kernel: {cp:.0f} GB/s; halo kernel at "
        f"{roof['frac_of_achievable']:.2f} of it")
    gbps_pay = value * h["payload_bytes"] / 1e9
    # line-granular bytes: a message's extent in whole 128-byte lines, read
    # on one side and written on the other
    extent = (h["count"] - 1) * 32 + 12
    line_bytes = 2 * (-(-extent // 128) * 128)
    hs = h.get("host_synced_msgs_per_s")
    line = {
        "metric": "enqueued msgs/s + GB/s (frac of HBM peak) vs host-synced path; p50/p99 latency",
        "value": value,
        "unit": "msgs/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"ring_halo_8ranks_vector(count={h['count']},bl=3,stride=8)_f32",
                   "ranks": n, "count": h["count"], "payload_bytes": h["payload_bytes"],
                   "msgs_per_step": 16, "parallelism": "1 GPU, 8 rank threads",
                   "variant": vname},
        "gbps_payload": gbps_pay,
        "gbps_algorithmic": 2 * gbps_pay,
        "gbps_line": value * line_bytes / 1e9,
        "hbm_frac": 2 * gbps_pay / HBM_PEAK_GBS,
        "plain_enqueue": {"value": h["msgs_per_s"], "ms_per_step": h["ms_per_step"],
                          "enqueue_ms_per_step": h["enqueue_ms_per_step"],
                          "p50_step_us": h["p50_step_us"], "p99_step_us": h["p99_step_us"]},
        "grouped_enqueue": {"value": h["grouped_msgs_per_s"], "ms_per_step": h["grouped_ms_per_step"],
                            "p50_step_us": h["grouped_p50_step_us"],
                            "p99_step_us": h["grouped_p99_step_us"]},
        "persistent_enqueue": {"value": h["persistent_msgs_per_s"],
                               "ms_per_step": h["persistent_ms_per_step"],
                               "p50_step_us": h["persistent_p50_step_us"],
                               "p99_step_us": h["persistent_p99_step_us"]},
        "host_synced": {"value": hs, "unit": "msgs/s", "speedup": value / hs if hs else None,
                        "plain_speedup": h["msgs_per_s"] / hs if hs else None},
        "latency_us": {"p50": h[k50], "p99": h[k99], "of": "halo step"},
        "roofline": roof,
        "sweep": out_sweep if args.sweep else None,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = halo_cpu_baseline(h["count"], args.cpu_budget)
    return line


# --------------------------------------------------------------- allreduce
def bench_allreduce(args):
    import numpy as np
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    from workloads import configs as C

    n = args.ranks
    nbytes = args.bytes
    dtype = args.dtype
    esize = {"int32": 4, "int64": 8, "float32": 4, "float64": 8}[dtype]
    count = nbytes // esize
    p = C.allreduce(nbytes, dtype, nranks=n, calls=1)
    S = [torch.from_numpy(p.buffers[r]["send"]).cuda() for r in range(n)]
    R = [torch.zeros(nbytes, dtype=torch.uint8, device="cuda") for _ in range(n)]
    torch.cuda.synchronize()

    def ops(k, marks=False):
        out = []
        for r in range(n):
            rows = []
            for s in range(k):
                if marks:
                    rows.append(dict(kind=D.MARK, req=2 * s))
                rows.append(dict(kind=D.ALLREDUCE, count=count, datatype=M.BASIC[dtype],
                                 op=M.SUM, buf=S[r].data_ptr(), buf2=R[r].data_ptr()))
                if marks:
                    rows.append(dict(kind=D.MARK, req=2 * s + 1))
            out.append(D.ops_array(rows))
        return out

    if args.group > 1 and args.group_only:
        # only the grouped comparison (e.g. under a profiler, without the
        # single-call passes)
        grouped = allreduce_groups(args, n, count, dtype, S, p)
        best = max((v for k, v in grouped.items() if k in ("plain", "grouped", "persistent")),
                   default=0.0)
        return {"metric": "enqueued allreduces/s, several per step", "value": best,
                "unit": "allreduces/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                "ms_per_step": 1000 * args.group / best if best else None, "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
                "config": {"workload": f"allreduce_sum_{n}ranks_{dtype}_{nbytes}B_x{args.group}",
                           "ranks": n, "bytes_per_rank": nbytes},
                "grouped": grouped}
    sess = D.Session(n)
    if args.via_host_synced:
        # counter collection serialises dispatches, which the cross-stream
        # device waits of the enqueue path cannot tolerate; the host-synced
        # path runs the same reduce kernel without them
        run_checked(sess, ops(args.warmup), mode=1)
        run_checked(sess, ops(args.steps), mode=1)
        close_checked(sess)
        return {"workload": f"allreduce_{n}r_{dtype}_{nbytes}B", "via": "host-synced"}
    run_checked(sess, ops(args.warmup))
    sec, _ = run_checked(sess, ops(args.steps))
    _, marks = run_checked(sess, ops(args.steps, True), nmarks=2 * args.steps)
    lat = step_latencies(marks, args.steps)
    # sampled check against the oracle's fold (every 4097th element), read
    # after the rank streams' own synchronisation
    from oracle import reduce as red
    idx = np.arange(0, count, 4097)
    ins = [np.frombuffer(p.buffers[r]["send"].tobytes(), dtype=dtype)[idx] for r in range(n)]
    want = red.fold("sum", ins)
    for r in (0, n - 1):
        got = np.frombuffer(R[r].cpu().numpy().tobytes(), dtype=dtype)[idx]
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), "allreduce != oracle"
    close_checked(sess)
    hs = None
    if not args.no_host_synced:
        sess = D.Session(n)
        run_checked(sess, ops(min(args.warmup, 3)), mode=1)
        k = max(1, min(args.steps, args.hs_steps))
        sec_hs, _ = run_checked(sess, ops(k), mode=1)
        close_checked(sess)
        hs = k / sec_hs
    grouped = allreduce_groups(args, n, count, dtype, S, p) if args.group > 1 else None
    cfg = M.Config()
    cfg.profile = 1
    sess = D.Session(n, cfg)
    run_checked(sess, ops(args.steps))
    torch.cuda.synchronize()
    st = sess.stats()
    close_checked(sess)
    avg_us = 1000 * st.reduce_ms / max(1, st.timed_reduce)
    per_launch = 2 * n * nbytes
    achieved = per_launch / (avg_us * 1e-6) / 1e9
    calls_per_s = args.steps / sec
    line = {
        "metric": "enqueued allreduce calls/s + GB/s (frac of HBM peak) vs host-synced path",
        "value": calls_per_s, "unit": "calls/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000 * sec / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"float32": "f32", "int64": "int64",
                                                          "int32": "int32", "float64": "f64"}[dtype],
        "data": "synthetic",
        "config": {"workload": f"allreduce_sum_{n}ranks_{dtype}_{nbytes}B_per_rank", "ranks": n,
                   "bytes_per_rank": nbytes},
        "gbps_algorithmic": per_launch * calls_per_s / 1e9,
        "hbm_frac": per_launch * calls_per_s / 1e9 / HBM_PEAK_GBS,
        "host_synced": {"value": hs, "unit": "calls/s",
                        "speedup": calls_per_s / hs if hs else None},
        "latency_us": {"p50": pct(lat, 50), "p99": pct(lat, 99), "of": "allreduce call"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(f"reduce_{n}x{nbytes >> 20}MiB_f32")
                     if dtype == "float32" else None,
                     "kernel": f"k_reduce<{dtype},SUM,vec>", "bytes_per_launch": per_launch,
                     "avg_launch_us": avg_us, "launches_timed": int(st.timed_reduce)},
    }
    if grouped:
        line["grouped"] = grouped
    return line


def allreduce_groups(args, n, count, dtype, S, p):
    """G allreduces per step (each on its own slice of the buffers) issued as
    G enqueue calls, as one group, as a persistent group started every step,
    and as G host-synchronised calls; allreduces per second."""
    import numpy as np
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    G = args.group
    nbytes = args.bytes
    S2 = [S[r].repeat(G) for r in range(n)]
    R2 = [torch.zeros(G * nbytes, dtype=torch.uint8, device="cuda") for _ in range(n)]
    torch.cuda.synchronize()

    def red(r, i):
        return dict(kind=D.ALLREDUCE, count=count, datatype=M.BASIC[dtype], op=M.SUM,
                    buf=S2[r].data_ptr() + i * nbytes, buf2=R2[r].data_ptr() + i * nbytes)

    def ops(variant, k):
        out = []
        for r in range(n):
            rows = []
            if variant == "init":
                rows = ([dict(kind=D.GROUP_START)] + [red(r, i) for i in range(G)]
                        + [dict(kind=D.GROUP_INIT, req=0)])
            elif variant == "persistent":
                rows = [dict(kind=D.BATCH_START, req=0) for _ in range(k)]
            else:
                for _ in range(k):
                    if variant == "grouped":
                        rows.append(dict(kind=D.GROUP_START))
                    rows += [red(r, i) for i in range(G)]
                    if variant == "grouped":
                        rows.append(dict(kind=D.GROUP_END))
            out.append(D.ops_array(rows))
        return out

    res = {}
    chosen = args.group_variants.split(",")
    for variant, mode in (("plain", 0), ("grouped", 0), ("persistent", 0), ("host", 1)):
        if variant == "host" and args.no_host_synced or variant not in chosen:
            continue
        k = args.steps if variant != "host" else max(1, min(args.steps, args.hs_steps))
        sess = D.Session(n)
        if variant == "persistent":
            run_checked(sess, ops("init", 0))
        run_checked(sess, ops(variant, min(args.warmup, 3)), mode=mode)
        secs = sorted(run_checked(sess, ops(variant, k), mode=mode)[0] for _ in range(3))
        res[variant] = G * k / secs[1]
        log(f"[allreduce x{G}] {variant}: {res[variant]:.0f} allreduces/s")
        # every slice holds the rank-order fold (sampled), read after the
        # rank streams' own synchronisation
        from oracle import reduce as redo
        idx = np.arange(0, count, 97)
        ins = [np.frombuffer(p.buffers[q]["send"].tobytes(), dtype=dtype)[idx] for q in range(n)]
        want = redo.fold("sum", ins).view(np.uint8)
        for r in (0, n - 1):
            got = R2[r].cpu().numpy().view(dtype).reshape(G, count)[:, idx]
            bad = [i for i in range(G)
                   if not np.array_equal(np.ascontiguousarray(got[i]).view(np.uint8), want)]
            if bad:
                raise AssertionError(f"{variant}: rank {r} slices {bad} differ from the oracle")
            R2[r].zero_()
        torch.cuda.current_stream().synchronize()
        close_checked(sess)
    return {"allreduces_per_step": G, "unit": "allreduces/s",
            **{f"{v}": res[v] for v in res},
            "grouped_vs_host": res["grouped"] / res["host"] if {"grouped", "host"} <= set(res) else None,
            "persistent_vs_host": (res["persistent"] / res["host"]
                                   if {"persistent", "host"} <= set(res) else None)}


# ------------------------------------------------------------------- batch
def bench_batch(args):
    """Config 4: 10,000 send/recv pairs over 32 ranks (sizes log-uniform
    8 B .. 256 KiB, tags 0..63, 30 % vector datatypes).  Each rank isends
    all its messages in global order, irecvs all of its messages, and waits
    for all of them.  Variants: one group per batch (one batch kernel), the
    plain enqueue path (one copy per message), and the host-synchronised path
    (blocking calls in global message order)."""
    import numpy as np
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    from workloads import configs as C
    from workloads.program import Recv, Send, Wait

    npairs, n = args.pairs, args.ranks_batch
    p = C.batch(npairs=npairs, nranks=n)
    msgs = C.batch_messages(npairs=npairs, nranks=n)
    types = {}

    def tt(tree):
        key = repr(tree)
        if key not in types:
            if isinstance(tree, str):
                types[key] = M.BASIC[tree]
            else:
                _, c, bl, st, base = tree
                types[key] = make_vector(M, c, bl, st, M.BASIC[base])
        return types[key]

    S = [torch.from_numpy(p.buffers[r]["sbuf"]).cuda() for r in range(n)]
    R = {v: [torch.from_numpy(p.buffers[r]["rbuf"].copy()).cuda() for r in range(n)]
         for v in ("persistent", "grouped", "plain", "host", "tune")}
    torch.cuda.synchronize()
    maxreq = max(len(p.ops[r][0]) for r in range(n)) + 1

    def ops(variant, reps, tag_base=0, marks=False):
        out = []
        for r in range(n):
            rows = []
            if variant in ("persistent", "tune") and reps > 0:
                for j in range(reps):
                    if marks:
                        rows.append(dict(kind=D.MARK, req=2 * j))
                    rows.append(dict(kind=D.BATCH_START, req=0))
                    if marks:
                        rows.append(dict(kind=D.MARK, req=2 * j + 1))
                out.append(D.ops_array(rows))
                continue
            for _ in range(max(reps, 1)):
                if variant in ("grouped", "persistent", "tune"):
                    rows.append(dict(kind=D.GROUP_START))
                if variant in ("grouped", "plain", "persistent", "tune"):
                    nreq = 0
                    for o in p.ops[r][0]:
                        if isinstance(o, Send):
                            rows.append(dict(kind=D.ISEND, peer=o.dest, tag=tag_base + o.tag,
                                             count=o.count, datatype=tt(o.dtype),
                                             buf=S[r].data_ptr() + o.off, req=nreq))
                            nreq += 1
                        elif isinstance(o, Recv):
                            rows.append(dict(kind=D.IRECV, peer=o.source, tag=tag_base + o.tag,
                                             count=o.count, datatype=tt(o.dtype),
                                             buf=R[variant][r].data_ptr() + o.off, req=nreq))
                            nreq += 1
                        elif isinstance(o, Wait):
                            rows.append(dict(kind=D.WAITALL, req=0, nreq=nreq))
                if variant == "grouped":
                    rows.append(dict(kind=D.GROUP_END))
                if variant in ("persistent", "tune"):
                    rows.append(dict(kind=D.GROUP_INIT, req=0))
                if variant == "host":
                    # blocking calls in global message order (deadlock-free)
                    sends = [o for o in p.ops[r][0] if isinstance(o, Send)]
                    recvs = [o for o in p.ops[r][0] if isinstance(o, Recv)]
                    si = ri = 0
                    for m in msgs:
                        if m["src"] == r:
                            o = sends[si]
                            si += 1
                            rows.append(dict(kind=D.SEND, peer=o.dest, tag=tag_base + o.tag,
                                             count=o.count, datatype=tt(o.dtype),
                                             buf=S[r].data_ptr() + o.off))
                        elif m["dst"] == r:
                            o = recvs[ri]
                            ri += 1
                            rows.append(dict(kind=D.RECV, peer=o.source, tag=tag_base + o.tag,
                                             count=o.count, datatype=tt(o.dtype),
                                             buf=R["host"][r].data_ptr() + o.off))
            out.append(D.ops_array(rows))
        return out

    # schedule of the persistent batch: chosen by the autotuner, or given
    sched = dict(tile=args.batch_tile, max_wg=args.batch_max_wg, graph=args.batch_graph,
                 sync=args.batch_sync)
    if args.kernel_only:
        # counter runs: plan the batch (no GPU waits) and launch its kernel only
        from paper_2208_13707_amd import tune
        sess = D.Session(n, tune.config_for(sched["tile"], sched["max_wg"], sched["graph"],
                                            nontemporal=args.batch_nt, sync=sched["sync"]))
        run_checked(sess, ops("persistent", 0), max_reqs=maxreq)
        us, payload, nwg = time_batch_kernel(sess, args.steps)
        close_checked(sess)
        return {"workload": "batch kernel only", "avg_launch_us": us, "payload_bytes": payload,
                "workgroups": nwg, "launches": args.steps + 1}
    tuned = None
    if args.tune and not args.only_grouped:
        from paper_2208_13707_amd import tune
        best, rows = tune.tune_batch(n, lambda: ops("tune", 0), lambda k: ops("tune", k),
                                     runs=max(20, args.steps), warm=3, max_reqs=maxreq, log=log)
        sched = {k: best[k] for k in ("tile", "max_wg", "graph", "sync")}
        tuned = {"chosen": best, "grid": rows}

    res = {}
    init_ms = None
    for variant, mode, tagb in (("persistent", 0, 2000), ("grouped", 0, 1000), ("plain", 0, 0),
                                ("host", 1, 0)):
        if variant == "host" and args.no_host_synced:
            continue
        if args.only_grouped and variant not in ("grouped", "persistent"):
            continue
        k = args.steps if variant != "host" else max(1, min(args.steps, args.hs_steps))
        cfg = None
        if variant == "persistent":
            from paper_2208_13707_amd import tune
            cfg = tune.config_for(sched["tile"], sched["max_wg"], sched["graph"],
                                  nontemporal=args.batch_nt, sync=sched["sync"])
        sess = D.Session(n, cfg)
        if variant == "persistent":
            init_ms = 1000 * run_checked(sess, ops(variant, 0, tagb), max_reqs=maxreq)[0]
        run_checked(sess, ops(variant, args.warmup, tagb), mode=mode, max_reqs=maxreq)
        sess.reset_stats()
        # median of three timings for the fast variants
        reps = 3 if variant in ("persistent", "grouped") else 1
        secs = sorted(run_checked(sess, ops(variant, k, tagb), mode=mode, max_reqs=maxreq)[0]
                      for _ in range(reps))
        sec = secs[len(secs) // 2]
        st = sess.stats()
        log(f"[batch] {variant}: host waits {st.host_waits}, sleeps {st.host_sleeps}, "
            f"sleep timeouts {st.host_sleep_timeouts} over {reps * k} batches, "
            f"{st.groups_planned} plans in {st.plan_ms:.1f} ms")
        if variant == "persistent":
            bk = time_batch_kernel(sess, 20)
            log(f"[batch] persistent: batch kernel alone {bk[0]:.1f} us")
            # per-batch latency: HIP events around every start on every stream
            _, mk = run_checked(sess, ops(variant, k, tagb, marks=True), max_reqs=maxreq,
                                nmarks=2 * k)
            lat = step_latencies(mk, k)
        close_checked(sess)
        if variant == "persistent" and args.trace:
            # a traced session of its own: where each run's time goes
            cfg.trace_events = 1 << 15
            ts = D.Session(n, cfg)
            run_checked(ts, ops(variant, 0, tagb), max_reqs=maxreq)
            ts_sec = run_checked(ts, ops(variant, k, tagb), max_reqs=maxreq)[0]
            tr = batch_trace_breakdown(M, ts.world, min(1 << 15, 96 * n * k))
            close_checked(ts)
            tr["ms_per_batch_traced"] = 1000 * ts_sec / k
            log(f"[batch] persistent trace: {json.dumps(tr)}")
        res[variant] = npairs * k / sec
        log(f"[batch] {variant}: {res[variant]:.0f} msgs/s ({1000 * sec / k:.3f} ms per batch)")
    if args.only_grouped:
        return {"workload": "batch", "grouped_msgs_per_s": res["grouped"],
                "persistent_msgs_per_s": res["persistent"]}
    # identical results across the paths and the oracle (on a sampled set of ranks)
    for v in res:
        for r in range(n):
            if not torch.equal(R[v][r], R["grouped"][r]):
                raise AssertionError(f"{v} path differs from grouped on rank {r}")
    head = res["persistent"]
    bk_us, bk_payload, bk_wg = bk
    per_launch = 2 * bk_payload
    gbps_alg = per_launch * head / npairs / 1e9
    line = {
        "metric": "enqueued msgs/s + GB/s (frac of HBM peak) vs host-synced path; p50/p99 latency",
        "value": head, "unit": "msgs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000 * npairs / head,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"batch_{npairs}pairs_{n}ranks_8B-256KiB_30pct_vector",
                   "ranks": n, "pairs": npairs, "payload_bytes_per_batch": bk_payload,
                   "variant": "persistent batch: planned once, one batch kernel per step",
                   "schedule": sched},
        "gbps_algorithmic": gbps_alg,
        "hbm_frac": gbps_alg / HBM_PEAK_GBS,
        "latency_us": {"p50": pct(lat, 50), "p99": pct(lat, 99), "of": "batch (10,000 messages)"},
        "persistent_init_ms": init_ms,
        "one_shot_group": {"value": res["grouped"], "unit": "msgs/s"},
        "plain_enqueue": {"value": res["plain"], "unit": "msgs/s"},
        "host_synced": {"value": res.get("host"), "unit": "msgs/s",
                        "speedup": head / res["host"] if "host" in res else None,
                        "one_shot_group_speedup": res["grouped"] / res["host"] if "host" in res else None,
                        "plain_speedup": res["plain"] / res["host"] if "host" in res else None},
    }
    ach = per_launch / (bk_us * 1e-6) / 1e9
    rates = pattern_rates(log_rows=True)
    bound = pattern_bound_us(msgs, rates)
    line["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic("batch_10000", bk_wg),
                        "pattern_bound_us": bound,
                        "frac_of_pattern_bound": bound / bk_us,
                        "pattern_rates_TBps": {str(k): v for k, v in rates.items()},
                        "kernel": f"mpixs::k_batch<{sched['tile']}, "
                                  f"{'true' if batch_nt_used(args.batch_nt, bk_payload) else 'false'}>",
                        "bytes_per_launch": per_launch, "avg_launch_us": bk_us,
                        "launches_timed": 20, "workgroups": bk_wg,
                        "note": "batch kernel of the whole 10,000-message group, launched back "
                                "to back between one event pair"}
    if tuned:
        line["autotune"] = tuned
    if not args.no_cpu_baseline:
        from oracle import simulate as sim
        # the whole batch through the oracle, repeated until about 10 s of
        # CPU work (the first result also checks the GPU's)
        t0 = time.perf_counter()
        ref = sim.run(p)
        runs = 1
        while time.perf_counter() - t0 < 10.0 and runs < 8:
            sim.run(p)
            runs += 1
        dt = time.perf_counter() - t0
        for r in range(n):
            if not np.array_equal(R["grouped"][r].cpu().numpy(), ref.buffers[r]["rbuf"]):
                raise AssertionError(f"rank {r}: batch result differs from the oracle")
        line["cpu_baseline"] = {"value": runs * npairs / dt, "unit": "msgs/s", "cores": 1,
                                "kind": "oracle",
                                "gbps_algorithmic": runs * 2 * bk_payload / dt / 1e9,
                                "sample": f"the whole batch ({npairs} messages) {runs} times, "
                                          f"{dt:.1f} s"}
    return line


# ------------------------------------------------------------------- serve
def bench_serve(args):
    """Config 5: 64 rank threads serve an open-loop Poisson stream of
    requests (60 % send/recv, 30 % isend+wait, 10 % allreduce-sum int32 over
    all ranks; bytes log-uniform 64 B .. 4 MiB) admitted under an 8 GB device
    budget; arrival rate swept 1e4 .. 1e6 per second.  Each rate is served
    again through the host-synchronised calls on the same schedule, whose
    results must be identical."""
    import numpy as np
    from paper_2208_13707_amd import driver as D
    from workloads import configs as C
    from workloads import payload

    n = args.serve_ranks
    sess = D.Session(n)
    rates = [float(x) for x in args.serve_rates.split(",")]
    sums = D.SERVE_RANK0_SUM if args.serve_sums == "rank0" else 0
    rows = []
    try:
        rc, _, _ = sess.serve(C.serving_schedule(1e4, 64, nranks=n, seed=99), args.budget,
                              flags=sums)
        if rc:
            raise RuntimeError(f"serve warm-up failed: {rc}")
        for k, rate in enumerate(rates):
            nreq = int(min(args.serve_max, max(200, rate * args.serve_seconds)))
            sched = C.serving_schedule(rate, nreq, nranks=n, seed=k + 1)
            rc, res, wall = sess.serve(sched, args.budget, flags=sums)
            if rc:
                raise RuntimeError(f"serve at rate {rate:g}: error {rc}")
            arr = np.array([q["arrival_us"] for q in sched])
            lat = res["done_us"] - arr
            wait = res["admit_us"] - arr
            # sampled check of results: payloads are regenerated on the host
            # from their published definition; an allreduce's expected output
            # is the int32 sum (wrapping) of its ranks' payloads -- checked
            # for up to three allreduces of at most 256 KiB per rate
            def wsum(b):
                j = np.arange(1, b.size + 1, dtype=np.uint64)
                with np.errstate(over="ignore"):
                    return int((b.astype(np.uint64) * j).sum(dtype=np.uint64))
            n_ar = 0
            for i in list(range(0, nreq, max(1, nreq // 50))) + \
                    [k for k, q in enumerate(sched) if q["kind"] == 2 and q["bytes"] <= 1 << 18]:
                q = sched[i]
                if q["kind"] == 2:
                    if q["bytes"] > 1 << 18 or n_ar >= 3:
                        continue
                    n_ar += 1
                    acc = np.zeros(q["bytes"] // 4, dtype=np.int32)
                    with np.errstate(over="ignore"):
                        for r in range(n):
                            acc += payload.fill(q["seed"] + r, q["bytes"]).view(np.int32)
                    # every rank's output is the sum: rank r weighted 2r + 1
                    want = wsum(acc.view(np.uint8)) * (1 if sums else n * n) % (1 << 64)
                else:
                    want = wsum(payload.fill(q["seed"], q["bytes"]))
                if int(res["checksum"][i]) != want:
                    raise AssertionError(f"request {i}: checksum differs")
            row = {"offered_per_s": rate, "requests": nreq,
                   "served_per_s": nreq / wall if wall > 0 else None,
                   "p50_latency_us": pct(lat, 50), "p99_latency_us": pct(lat, 99),
                   "p99_admission_wait_us": pct(wait, 99),
                   "gbps_payload": float(sum(q["bytes"] * (n if q["kind"] == 2 else 1)
                                             for q in sched)) / wall / 1e9}
            if not args.no_host_synced:
                # the comparison path on the same schedule: host-synchronised
                # calls, every checksum equal to the enqueue path's
                rc, hres, hwall = sess.serve(sched, args.budget, flags=sums | D.SERVE_HOST_SYNCED)
                if rc:
                    raise RuntimeError(f"host-synced serve at rate {rate:g}: error {rc}")
                if not np.array_equal(hres["checksum"], res["checksum"]):
                    raise AssertionError(f"rate {rate:g}: host-synced results differ")
                hlat = hres["done_us"] - arr
                hs = nreq / hwall if hwall > 0 else None
                row["host_synced"] = {"served_per_s": hs, "p50_latency_us": pct(hlat, 50),
                                      "p99_latency_us": pct(hlat, 99)}
                row["speedup"] = (row["served_per_s"] / hs) if hs else None
            rows.append(row)
            log(f"[serve] offered {rate:9.0f}/s: served {row['served_per_s']:9.0f}/s, "
                f"p50 {row['p50_latency_us']:8.1f} us, p99 {row['p99_latency_us']:9.1f} us"
                + (f"; host-synced {row['host_synced']['served_per_s']:9.0f}/s, "
                   f"p50 {row['host_synced']['p50_latency_us']:8.1f} us, "
                   f"p99 {row['host_synced']['p99_latency_us']:9.1f} us"
                   if "host_synced" in row else ""))
    finally:
        close_checked(sess)
    best = max(rows, key=lambda r: r["served_per_s"] or 0)
    hs_rates = [r["host_synced"]["served_per_s"] or 0 for r in rows if "host_synced" in r]
    hs_best = max(hs_rates) if hs_rates else None
    return {
        "metric": "served requests/s with p50/p99 latency (open-loop Poisson arrivals)",
        "value": best["served_per_s"], "unit": "requests/s", "n_gpus": 1,
        "steps": sum(r["requests"] for r in rows), "warmup": 64,
        "ms_per_step": 1000.0 / best["served_per_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"serving_{n}ranks_mix60-30-10_64B-4MiB",
                   "budget_bytes": args.budget},
        "host_synced": {"value": hs_best, "unit": "requests/s",
                        "speedup": (best["served_per_s"] / hs_best) if hs_best else None},
        "checked": ("sampled point-to-point requests and up to 3 allreduces of <= 256 KiB per "
                    "rate against host-computed checksums (allreduce outputs checksummed on "
                    + ("rank 0" if sums else "every rank") + "); host-synchronised results "
                    "equal to the enqueue path's"),
        "sweep": rows,
    }


# ------------------------------------------------------------------ N-to-1
def bench_nto1(args):
    """N-to-1 through a multiplex stream communicator (§3.5): rank 0 runs
    N sender threads, each on its own stream, that isend M 8-byte messages
    per step to the single polling thread of rank 1, which receives them all
    on one communicator with ANY_INDEX / ANY_TAG.  Compared with N separate
    stream communicators (the polling thread addresses each in turn) and
    with the host-synchronised calls on those."""
    import numpy as np
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M

    n, per, steps, warm = args.nto1_senders, args.nto1_per_step, args.steps, args.warmup
    S = [torch.arange(2 * per, dtype=torch.int32, device="cuda") + 1000 * (i + 1)
         for i in range(n)]
    R = {v: torch.zeros(2 * n * per, dtype=torch.int32, device="cuda")
         for v in ("mux", "pairs", "host")}
    torch.cuda.synchronize()
    dt = M.BASIC["int32"]

    def ops(variant, k):
        senders, recv = [], []
        for i in range(n):
            rows = []
            for _ in range(k):
                for j in range(per):
                    a = S[i].data_ptr() + 8 * j
                    if variant == "mux":
                        rows.append(dict(kind=D.STREAM_ISEND, comm=0, peer=1, tag=j, count=2,
                                         datatype=dt, buf=a, req=j, op=i, pad=0))
                    elif variant == "pairs":
                        rows.append(dict(kind=D.ISEND, comm=1, peer=1, tag=j, count=2,
                                         datatype=dt, buf=a, req=j))
                    else:
                        rows.append(dict(kind=D.SEND, comm=1, peer=1, tag=j, count=2,
                                         datatype=dt, buf=a))
                if variant != "host":
                    rows.append(dict(kind=D.WAITALL, req=0, nreq=per))
            senders.append(D.ops_array(rows))
        rows = []
        for _ in range(k):
            slot = 0
            for j in range(per):
                for i in range(n):
                    a = R[variant].data_ptr() + 8 * (j * n + i)
                    if variant == "mux":
                        rows.append(dict(kind=D.STREAM_IRECV, comm=0, peer=M.ANY_SOURCE,
                                         tag=M.ANY_TAG, count=2, datatype=dt, buf=a, req=slot,
                                         op=M.ANY_INDEX, pad=0))
                    elif variant == "pairs":
                        rows.append(dict(kind=D.IRECV, comm=1 + i, peer=0, tag=j, count=2,
                                         datatype=dt, buf=a, req=slot))
                    else:
                        rows.append(dict(kind=D.RECV, comm=1 + i, peer=0, tag=j, count=2,
                                         datatype=dt, buf=a))
                    slot += 1
            if variant != "host":
                rows.append(dict(kind=D.WAITALL, req=0, nreq=slot))
        return senders, D.ops_array(rows)

    res = {}
    for variant, mode in (("mux", 0), ("pairs", 0), ("host", 1)):
        if variant == "host" and args.no_host_synced:
            continue
        sess = D.NTo1Session(n)
        k = steps if variant != "host" else max(1, min(steps, args.hs_steps))
        s_ops, r_ops = ops(variant, warm)
        rc, r, _ = sess.run(s_ops, r_ops, mode=mode, max_reqs=n * per)
        if rc:
            raise RuntimeError(f"nto1 {variant}: {M.errname(rc)}")
        s_ops, r_ops = ops(variant, k)
        rc, r, _ = sess.run(s_ops, r_ops, mode=mode, max_reqs=n * per)
        if rc:
            raise RuntimeError(f"nto1 {variant}: {M.errname(rc)}")
        if variant == "mux":
            # one more step into a cleared buffer: across steps a wildcard
            # receive may take a fast sender's next-step message, so the
            # exact check is made on a single step, where every message
            # meets exactly one of the step's receives
            R["mux"].zero_()
            torch.cuda.current_stream().synchronize()
            s_ops, r_ops = ops(variant, 1)
            rc, _, _ = sess.run(s_ops, r_ops, mode=mode, max_reqs=n * per)
            if rc:
                raise RuntimeError(f"nto1 {variant}: {M.errname(rc)}")
            # each runner thread synchronised its own stream
            want = np.sort(np.concatenate([s.cpu().numpy() for s in S]))
            if not np.array_equal(np.sort(R["mux"].cpu().numpy()), want):
                raise AssertionError("multiplex N-to-1 lost or duplicated a message")
        close_checked(sess)
        res[variant] = n * per * k / r.seconds
        log(f"[nto1] {variant}: {res[variant]:.0f} msgs/s")
    if "host" in res and not torch.equal(R["pairs"], R["host"]):
        raise AssertionError("N-to-1 over pairs differs from the host-synchronised path")
    return {
        "metric": "enqueued msgs/s, N-to-1 over one multiplex communicator (8-byte messages)",
        "value": res["mux"], "unit": "msgs/s", "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": 1000.0 * n * per / res["mux"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
        "config": {"workload": f"n_to_1_{n}senders_{per}msgs_per_step_8B"},
        "separate_stream_comms": {"value": res["pairs"], "unit": "msgs/s"},
        "host_synced": {"value": res.get("host"), "unit": "msgs/s",
                        "speedup": res["mux"] / res["host"] if "host" in res else None},
    }


# ---------------------------------------------------------------- hostrate
def bench_hostrate(args):
    """CPU only: the host message-rate model under the three engine policies
    (global critical section, per-context critical sections, stream contexts),
    8-byte isend / irecv in windows of 64, 1..P thread pairs; best of 3."""
    from paper_2208_13707_amd import driver as D
    cpus = len(os.sched_getaffinity(0))
    pairs = [p for p in (1, 2, 4, 8, 16) if 2 * p <= cpus] or [1]
    per = args.hostrate_msgs
    want = {}
    curves = {}
    for pol in ("global", "per_context", "stream"):
        curves[pol] = []
        for p in pairs:
            best = 0.0
            for _ in range(3):
                rc, rate, ck = D.mpixs_drv_host_msgrate(p, pol, per, 64)
                if rc:
                    raise RuntimeError(f"host_msgrate({p}, {pol}): rc {rc}")
                if want.setdefault(p, ck) != ck:
                    raise AssertionError(f"host_msgrate checksum differs ({p} pairs, {pol})")
                best = max(best, rate)
            curves[pol].append(best)
            log(f"[hostrate] {pol} {p} pairs: {best / 1e6:.2f} M msgs/s")
    top = curves["stream"][-1]
    return {
        "metric": "host message rate, 8-byte isend/irecv (CPU model, no GPU)",
        "value": top, "unit": "msgs/s", "n_gpus": 0, "steps": per, "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"host_msgrate_{pairs[-1]}pairs_window64_{per}msgs_per_pair",
                   "thread_pairs": pairs, "cpus": cpus},
        "curves_msgs_per_s": curves,
        "stream_vs_per_context": [s / v for s, v in zip(curves["stream"], curves["per_context"])],
    }


# ---------------------------------------------------------------- pingpong
def trace_breakdown(M, world, cap):
    """Per-message step times from the device trace: the events of one
    message share its channel block and counter value (POST and MATCH on the
    first side's ready word, DONE and COMPLETE on done); p50/p99 of
    POST -> MATCH (the other side reaching the message after it was posted),
    MATCH -> DONE (the copy) and DONE -> COMPLETE (the first side seeing it),
    in microseconds of device time."""
    from collections import defaultdict
    rc, total, ev = M.mpixs_world_trace(world, cap)
    if rc:
        raise RuntimeError(f"mpixs_world_trace: {M.errname(rc)}")
    groups = defaultdict(dict)
    for e in ev:
        groups[(e.counter & ~63, e.value)].setdefault(e.kind, e)
    steps = {"post_to_match_us": [], "match_to_done_us": [], "done_to_complete_us": []}
    eager = 0
    for g in groups.values():
        if set(g) == {M.TRACE_POST, M.TRACE_MATCH, M.TRACE_DONE, M.TRACE_COMPLETE}:
            t = [g[k].time_ns for k in (M.TRACE_POST, M.TRACE_MATCH, M.TRACE_DONE,
                                        M.TRACE_COMPLETE)]
            for name, a, b in (("post_to_match_us", 0, 1), ("match_to_done_us", 1, 2),
                               ("done_to_complete_us", 2, 3)):
                steps[name].append((t[b] - t[a]) / 1000.0)
        elif set(g) == {M.TRACE_MATCH, M.TRACE_DONE}:
            eager += 1      # an eager send's staged copy (its pack is a DONE of its own)
    out = {"events": total, "messages": len(steps["post_to_match_us"]), "eager_copies": eager}
    for name, xs in steps.items():
        out[name] = {"p50": pct(xs, 50), "p99": pct(xs, 99)}
    return out


def batch_trace_breakdown(M, world, cap):
    """Per-run step times of a persistent batch from the device trace.  Run e
    leaves: every other rank's arrival (POST on its arrival word, value e),
    the launching rank's wait seeing each arrival (MATCH, same word and
    value), the signal after the batch kernel (DONE on the done word, value
    e) and every other rank's wait seeing it (COMPLETE, done word, value e).
    p50 / p99 over runs of (device microseconds):
    period (DONE of e-1 to DONE of e), others' turn (DONE of e-1 to the last
    POST of e: the other ranks' waits and next arrivals), launch wait (last
    POST to last MATCH), kernel (last MATCH to DONE: the batch kernel and the
    signal), and per other rank DONE -> COMPLETE and COMPLETE -> its next
    POST."""
    from collections import defaultdict
    rc, total, ev = M.mpixs_world_trace(world, cap)
    if rc:
        raise RuntimeError(f"mpixs_world_trace: {M.errname(rc)}")
    by = defaultdict(lambda: defaultdict(list))
    for e in ev:
        by[e.value][e.kind].append(e)
    done = {v: k[M.TRACE_DONE][0].time_ns for v, k in by.items() if len(k[M.TRACE_DONE]) == 1}
    cols = {k: [] for k in ("period_us", "others_turn_us", "launch_wait_us", "kernel_us",
                            "done_to_complete_us", "complete_to_next_post_us")}
    runs = 0
    for v in sorted(done):
        k = by[v]
        if v - 1 not in done or not k[M.TRACE_POST] or not k[M.TRACE_MATCH]:
            continue
        runs += 1
        last_post = max(e.time_ns for e in k[M.TRACE_POST])
        last_match = max(e.time_ns for e in k[M.TRACE_MATCH])
        cols["period_us"].append((done[v] - done[v - 1]) / 1e3)
        cols["others_turn_us"].append((last_post - done[v - 1]) / 1e3)
        cols["launch_wait_us"].append((last_match - last_post) / 1e3)
        cols["kernel_us"].append((done[v] - last_match) / 1e3)
        prev = by[v - 1]
        comp = {e.stream: e.time_ns for e in prev[M.TRACE_COMPLETE]}
        for e in prev[M.TRACE_COMPLETE]:
            cols["done_to_complete_us"].append((e.time_ns - done[v - 1]) / 1e3)
        for e in k[M.TRACE_POST]:
            if e.stream in comp:
                cols["complete_to_next_post_us"].append((e.time_ns - comp[e.stream]) / 1e3)
    out = {"events": total, "runs": runs}
    for name, xs in cols.items():
        out[name] = {"p50": pct(xs, 50), "p99": pct(xs, 99)}
    return out


def bench_pingpong(args):
    import numpy as np
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    from workloads import configs as C

    nmsg = 1000
    p = C.pingpong(nmsg=2)
    X = [torch.from_numpy(p.buffers[r]["x"].copy()).cuda() for r in range(2)]
    torch.cuda.synchronize()

    def ops(rounds, mode, marks=False):
        r0, r1 = [], []
        for s in range(rounds):
            if marks:
                r0.append(dict(kind=D.MARK, req=2 * s))
            r0 += [dict(kind=D.SEND, peer=1, tag=0, count=1024, datatype=M.INT32, buf=X[0].data_ptr()),
                   dict(kind=D.RECV, peer=1, tag=0, count=1024, datatype=M.INT32, buf=X[0].data_ptr())]
            if marks:
                r0.append(dict(kind=D.MARK, req=2 * s + 1))
            r1 += [dict(kind=D.RECV, peer=0, tag=0, count=1024, datatype=M.INT32, buf=X[1].data_ptr()),
                   dict(kind=D.SEND, peer=0, tag=0, count=1024, datatype=M.INT32, buf=X[1].data_ptr())]
        return [D.ops_array(r0), D.ops_array(r1)]

    out = {}
    for mode in (0, 1):
        if mode == 1 and args.no_host_synced:
            continue
        sess = D.Session(2)
        run_checked(sess, ops(20, mode), mode=mode)
        sec, _ = run_checked(sess, ops(nmsg // 2, mode), mode=mode)
        if mode == 0:
            _, marks = run_checked(sess, ops(nmsg // 2, mode, True), mode=mode, nmarks=nmsg)
            rtt = [(marks[0, 2 * s + 1] - marks[0, 2 * s]) * 1000 for s in range(nmsg // 2)]
            out["one_way_p50_us"] = pct(rtt, 50) / 2
            out["one_way_p99_us"] = pct(rtt, 99) / 2
        close_checked(sess)
        out[mode] = nmsg / sec
    if args.trace:
        # a separate traced pass: the per-message step times on the device
        cfg = M.Config()
        cfg.trace_events = 8 * nmsg
        sess = D.Session(2, cfg)
        run_checked(sess, ops(nmsg // 2, 0))
        out["trace"] = trace_breakdown(M, sess.world, 8 * nmsg)
        close_checked(sess)
        log(f"[pingpong] trace: {json.dumps(out['trace'])}")
    assert np.array_equal(X[0].cpu().numpy(), p.buffers[0]["x"]), "echo changed the data"
    return {
        "metric": "enqueued msgs/s vs host-synced path; p50/p99 one-way latency",
        "value": out[0], "unit": "msgs/s", "n_gpus": 1, "steps": nmsg, "warmup": 40,
        "ms_per_step": 1000 / out[0], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "pingpong_2ranks_1000x1024_int32"},
        "host_synced": {"value": out.get(1), "unit": "msgs/s",
                        "speedup": out[0] / out[1] if 1 in out else None},
        "latency_us": {"p50": out["one_way_p50_us"], "p99": out["one_way_p99_us"],
                       "of": "one-way (round trip / 2)"},
        "trace": out.get("trace"),
    }


# -------------------------------------------------------------------- copy
def achievable_copy_gbps(nbytes=1 << 30, launches=5):
    """HBM bandwidth the library's own copy kernel reaches on this GPU: one
    contiguous message of ``nbytes`` between two ranks, each launch timed
    with a HIP event pair on its stream (algorithmic bytes 2 x nbytes)."""
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    ops = lambda k: [D.ops_array([dict(kind=D.SEND, peer=1, tag=7, count=nbytes,
                                       datatype=M.UINT8, buf=src.data_ptr())] * k),
                     D.ops_array([dict(kind=D.RECV, peer=0, tag=7, count=nbytes,
                                       datatype=M.UINT8, buf=dst.data_ptr())] * k)]
    cfg = M.Config()
    cfg.profile = 1
    sess = D.Session(2, cfg)
    run_checked(sess, ops(2))
    sess.reset_stats()
    run_checked(sess, ops(launches))
    st = sess.stats()
    close_checked(sess)
    if not torch.equal(src, dst):
        raise AssertionError("copy calibration: destination differs from source")
    avg_us = 1000 * st.copy_ms / max(1, st.timed_copy)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (avg_us * 1e-6) / 1e9


def bench_copy(args):
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M

    nbytes = args.bytes
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()

    def ops(k):
        r0 = [dict(kind=D.SEND, peer=1, tag=7, count=nbytes, datatype=M.UINT8, buf=src.data_ptr())
              for _ in range(k)]
        r1 = [dict(kind=D.RECV, peer=0, tag=7, count=nbytes, datatype=M.UINT8, buf=dst.data_ptr())
              for _ in range(k)]
        return [D.ops_array(r0), D.ops_array(r1)]

    cfg = M.Config()
    cfg.profile = 1 if args.profile_copy else 0
    sess = D.Session(2, cfg)
    if args.via_host_synced:
        run_checked(sess, ops(args.warmup), mode=1)
        run_checked(sess, ops(args.steps), mode=1)
        close_checked(sess)
        return {"workload": f"send_recv_contiguous_{nbytes}B_2ranks", "via": "host-synced"}
    run_checked(sess, ops(args.warmup))
    sess.reset_stats()
    sec, _ = run_checked(sess, ops(args.steps))
    torch.cuda.synchronize()
    st = sess.stats()
    close_checked(sess)
    assert torch.equal(src, dst)
    gbps = 2 * nbytes * args.steps / sec / 1e9
    line = {
        "metric": "contiguous message GB/s (frac of HBM peak)", "value": gbps, "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000 * sec / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"send_recv_contiguous_{nbytes}B_2ranks"},
        "hbm_frac": gbps / HBM_PEAK_GBS,
    }
    if args.profile_copy:
        avg_us = 1000 * st.copy_ms / max(1, st.timed_copy)
        ach = 2 * nbytes / (avg_us * 1e-6) / 1e9
        line["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": ach / HBM_PEAK_GBS,
                            "traffic": measured_traffic("copy_contiguous_1GiB")
                            if nbytes == 1 << 30 else None,
                            "kernel": "k_copy<16,CONTIG,CONTIG>", "bytes_per_launch": 2 * nbytes,
                            "avg_launch_us": avg_us, "launches_timed": int(st.timed_copy)}
    if args.sweep:
        line["sweep"] = copy_sweep(args)
    return line


def copy_sweep(args):
    """Contiguous 2-rank send / recv from 1 MiB to 1 GiB: the enqueue path's
    GB/s (blocking calls, about 4 GiB moved per size), its copy kernel's own
    time (HIP events around each launch, a run of its own) and the
    host-synchronised path's GB/s, as algorithmic bytes (2 x the message)
    and fractions of 8 TB/s; the sizes from 512 MiB on exceed the 256 MB
    Infinity Cache."""
    import torch
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    rows = []
    for nbytes in [1 << 20, 4 << 20, 16 << 20, 64 << 20, 256 << 20, 512 << 20, 1 << 30]:
        src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
        dst = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        steps = max(4, min(2000, (4 << 30) // nbytes))

        def ops(k):
            r0 = [dict(kind=D.SEND, peer=1, tag=7, count=nbytes, datatype=M.UINT8,
                       buf=src.data_ptr()) for _ in range(k)]
            r1 = [dict(kind=D.RECV, peer=0, tag=7, count=nbytes, datatype=M.UINT8,
                       buf=dst.data_ptr()) for _ in range(k)]
            return [D.ops_array(r0), D.ops_array(r1)]

        row = {"bytes": nbytes, "steps": steps}
        for mode, key in ((0, "enqueue_GBps"), (1, "host_synced_GBps")):
            sess = D.Session(2)
            run_checked(sess, ops(2), mode=mode)
            sec, _ = run_checked(sess, ops(steps), mode=mode)
            close_checked(sess)
            row[key] = 2 * nbytes * steps / sec / 1e9
        cfg = M.Config()
        cfg.profile = 1
        sess = D.Session(2, cfg)
        run_checked(sess, ops(min(steps, 200)))
        torch.cuda.synchronize()
        st = sess.stats()
        close_checked(sess)
        assert torch.equal(src, dst)
        kus = 1000 * st.copy_ms / max(1, st.timed_copy)
        row["kernel_us"] = kus
        row["kernel_GBps"] = 2 * nbytes / (kus * 1e-6) / 1e9
        row["kernel_frac"] = row["kernel_GBps"] / HBM_PEAK_GBS
        row["enqueue_frac"] = row["enqueue_GBps"] / HBM_PEAK_GBS
        log(f"[copy] {nbytes >> 20:5d} MiB: enqueue {row['enqueue_GBps']:7.0f} GB/s "
            f"({row['enqueue_frac']:.2f}), kernel {kus:8.1f} us ({row['kernel_frac']:.2f}), "
            f"host-synced {row['host_synced_GBps']:7.0f} GB/s")
        rows.append(row)
        del src, dst
    return rows


def extra_configs(args):
    """The allreduce configuration at 64 MiB per rank (float32 and int64), the
    ring-halo configuration (tag = step), each at its full size, and the
    serving configuration (64 ranks, 64 B .. 4 MiB, 8 GB budget) at an
    unsaturated and a saturating arrival rate, for the default line."""
    import copy
    out = {}
    ar = {}
    for dtype in ("float32", "int64"):
        a = copy.copy(args)
        a.workload, a.bytes, a.dtype, a.ranks, a.group = "allreduce", 64 << 20, dtype, 16, 1
        a.steps, a.warmup, a.hs_steps, a.via_host_synced = 20, 5, 20, False
        r = bench_allreduce(a)
        ar[dtype] = {"calls_per_s": r["value"], "gbps_algorithmic": r["gbps_algorithmic"],
                     "hbm_frac": r["hbm_frac"], "host_synced": r["host_synced"],
                     "latency_us": r["latency_us"], "roofline": r["roofline"]}
        log(f"[extra] allreduce 16 x 64 MiB {dtype}: {r['value']:.0f} calls/s, "
            f"HBM frac {r['hbm_frac']:.3f} (kernel {r['roofline']['frac']:.3f})")
    out["config3_allreduce_16ranks_64MiB"] = ar
    a = copy.copy(args)
    a.workload, a.count, a.steps, a.warmup, a.sweep = "halo", 43690, 100, 10, False
    a.no_cpu_baseline, a.hs_steps = True, 100
    h = bench_halo(a)
    out["config2_ring_halo_count43690"] = {
        "value": h["plain_enqueue"]["value"], "unit": "msgs/s",
        "variant": "plain enqueue (one copy per message, tag = step)",
        "plain_enqueue": h["plain_enqueue"], "grouped_enqueue": h["grouped_enqueue"],
        "persistent_enqueue": h["persistent_enqueue"],
        "host_synced": h["host_synced"],
        "plain_vs_host_synced": h["host_synced"]["plain_speedup"],
        # the plain path's rates as payload, algorithmic (2 x payload) and
        # line-granular bytes (the halo line's per-message ratios)
        "gbps_payload": h["plain_enqueue"]["value"] * h["config"]["payload_bytes"] / 1e9,
        "gbps_algorithmic": 2 * h["plain_enqueue"]["value"] * h["config"]["payload_bytes"] / 1e9,
        "gbps_line": h["plain_enqueue"]["value"] * h["gbps_line"] / h["value"] if h["value"] else None,
        # the plain path's data kernel: one message's typemap copy
        "roofline": vector_copy_roofline(43690, 100),
        "roofline_batch_kernel": h["roofline"]}
    log(f"[extra] halo plain enqueue {h['plain_enqueue']['value']:.0f} msgs/s, "
        f"host-synced {h['host_synced']['value']:.0f}")
    a = copy.copy(args)
    a.workload, a.serve_rates, a.serve_seconds = "serve", "1e4,1e6", 0.5
    sv = bench_serve(a)
    out["config5_serving_64ranks"] = {
        "value": sv["value"], "unit": "requests/s", "host_synced": sv["host_synced"],
        "budget_bytes": sv["config"]["budget_bytes"], "sweep": sv["sweep"],
        "checked": sv["checked"]}
    hs = sv["host_synced"]["value"]
    log(f"[extra] serving 64 ranks: {sv['value']:.0f} requests/s, host-synced "
        + (f"{hs:.0f}" if hs else "not run"))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--no-extras", action="store_true",
                    help="batch: leave out the allreduce and halo configurations")
    ap.add_argument("--workload", default="batch",
                    choices=["halo", "pingpong", "allreduce", "copy", "vcopy", "batch", "serve",
                             "nto1", "hostrate", "patterns"])
    ap.add_argument("--hostrate-msgs", type=int, default=1000000,
                    help="hostrate: messages per thread pair")
    ap.add_argument("--nto1-senders", type=int, default=8)
    ap.add_argument("--nto1-per-step", type=int, default=16)
    ap.add_argument("--serve-ranks", type=int, default=64)
    ap.add_argument("--serve-rates", default="1e4,3e4,1e5,3e5,1e6")
    ap.add_argument("--serve-seconds", type=float, default=0.5)
    ap.add_argument("--serve-max", type=int, default=20000)
    ap.add_argument("--trace", action="store_true",
                    help="pingpong: also a traced pass; halo: trace the plain path's timed "
                         "steps (per-message step times read from the device trace); batch: "
                         "a traced pass of the persistent batch (per-run step times)")
    ap.add_argument("--serve-sums", choices=["all", "rank0"], default="rank0",
                    help="serve: checksum rank 0's allreduce output (the harness's own "
                         "verification; 64 checksum kernels per allreduce cost about 40 %% "
                         "of the throughput) or every rank's")
    ap.add_argument("--budget", type=int, default=8 << 30)
    ap.add_argument("--pairs", type=int, default=10000)
    ap.add_argument("--only-grouped", action="store_true",
                    help="batch: persistent and one-shot group variants only")
    ap.add_argument("--kernel-only", action="store_true",
                    help="halo / batch: plan the persistent batch and time its kernel only "
                         "(no device waits: for counter runs)")
    ap.add_argument("--tune", action="store_true",
                    help="batch: pick the persistent batch schedule by a grid search first")
    ap.add_argument("--batch-tile", type=int, default=256)
    ap.add_argument("--batch-max-wg", type=int, default=32768)
    ap.add_argument("--batch-graph", type=int, default=0)
    ap.add_argument("--batch-nt", type=int, default=0,
                    help="batch kernel nontemporal accesses: 0 auto, 1 on, 2 off")
    ap.add_argument("--batch-sync", type=int, default=0,
                    help="persistent batches: 0 device counters, 1 HIP events")
    ap.add_argument("--ranks-batch", type=int, default=32)
    ap.add_argument("--count", type=int, default=43690)
    ap.add_argument("--fuse-max-bytes", type=int, default=None,
                    help="halo: mpixs_config.fuse_max_bytes of the plain enqueue path")
    ap.add_argument("--sweep", action="store_true",
                    help="halo: also the other four counts; copy: message sizes 1 MiB .. 1 GiB")
    ap.add_argument("--tune-plain", action="store_true",
                    help="halo: choose the plain path's fuse threshold by a grid search first")
    ap.add_argument("--bytes", type=int, default=None)
    ap.add_argument("--dtype", default="float32")
    ap.add_argument("--ranks", type=int, default=16)
    ap.add_argument("--group", type=int, default=1,
                    help="allreduce: also time this many allreduces per step as plain calls, "
                         "one group, a persistent group and host-synchronised calls")
    ap.add_argument("--group-variants", default="plain,grouped,persistent,host",
                    help="allreduce --group: which of the four ways to time")
    ap.add_argument("--group-only", action="store_true",
                    help="allreduce --group: skip the single-call passes")
    ap.add_argument("--hs-steps", type=int, default=100)
    ap.add_argument("--no-host-synced", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--profile-copy", action="store_true")
    ap.add_argument("--via-host-synced", action="store_true",
                    help="copy/allreduce: run only the host-synchronised path (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: ranks are host threads "
              "sharing one MI355X", file=sys.stderr)
        sys.exit(2)
    defaults = {"halo": (100, 10), "pingpong": (1000, 40), "allreduce": (20, 5), "copy": (10, 3),
                "vcopy": (100, 10), "batch": (20, 5), "serve": (1, 0), "patterns": (20, 1),
                "nto1": (200, 20), "hostrate": (1, 0)}
    k, w = defaults[args.workload]
    args.steps = args.steps or k
    args.warmup = args.warmup if args.warmup is not None else w
    if args.bytes is None:
        args.bytes = {"allreduce": 64 << 20, "copy": 1 << 30}.get(args.workload, 0)
    if args.workload == "hostrate":
        print(json.dumps(bench_hostrate(args)), flush=True)
        return
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "vcopy":
        line = {"workload": f"vector_copy_count{args.count}",
                "roofline": vector_copy_roofline(args.count, args.steps)}
    elif args.workload == "patterns":
        line = {"workload": "copy kernel per layout pattern, 128 MiB payload",
                "unit": "TB/s algorithmic", "rates": pattern_rates(log_rows=True)}
    else:
        fn = {"halo": bench_halo, "allreduce": bench_allreduce, "pingpong": bench_pingpong,
              "copy": bench_copy, "batch": bench_batch, "serve": bench_serve,
              "nto1": bench_nto1}[args.workload]
        line = fn(args)
        if args.workload == "batch" and not args.no_extras and not args.kernel_only \
                and not args.only_grouped:
            line.update(extra_configs(args))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
