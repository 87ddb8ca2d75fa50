"""Floating-point edge values through every reduce kernel, bit for bit.

Inputs mix, element by element: signed zeros (MIN / MAX ties between -0 and
+0 keep the earlier operand of the fold), subnormals (kept, not flushed),
+-Inf on one rank, values near the overflow threshold (sums and products
that overflow to Inf), and ordinary N(0,1) values; no element can produce a
NaN (whose payload bits are unpinned).  Every result must equal the oracle's
canonical-order fold in its bit patterns, through the fused kernel (small
reductions), the split kernel with the rank count known only at run time,
the kernel unrolled over 16 ranks, and the merged kernel of a group.

NaN inputs (quiet NaNs of random sign and payload, on rank 0 or on later
ranks) go through the same four kernels: MIN / MAX must equal the oracle bit
for bit (a comparison with a NaN is false, so the fold keeps rank 0's NaN and
passes over later ones), SUM / PROD must give a NaN exactly where the oracle
does, and equal bits everywhere else (IEEE-754 fixes no NaN payload).
"""
import sys

import numpy as np
import pytest

from oracle import reduce as redo
from oracle import simulate as sim
from tests.gpu_runner import compare, run_program
from workloads.program import Allreduce, GroupEnd, GroupStart, as_bytes, single_stream

OPS = ("sum", "prod", "min", "max")


def edge_inputs(dtype, nranks, count, seed):
    """Per-rank arrays; element i is of class i mod 6."""
    g = np.random.default_rng([220813707, 80, seed])
    t = np.dtype(dtype)
    fi = np.finfo(t)
    tiny = fi.smallest_subnormal
    big = fi.max / 4
    cls = np.arange(count) % 6
    inf_rank = g.integers(nranks, size=count)
    inf_sign = np.where(g.uniform(size=count) < 0.5, -1.0, 1.0)
    out = []
    for r in range(nranks):
        x = g.standard_normal(count).astype(t)
        sign = np.where(g.uniform(size=count) < 0.5, -1.0, 1.0).astype(t)
        zeros = (sign * t.type(0.0)).astype(t)
        subn = (sign * g.integers(1, 1 << 20, size=count).astype(t) * tiny).astype(t)
        near = (sign * big * (1 + g.uniform(size=count))).astype(t)
        x = np.where(cls == 0, zeros, x)
        x = np.where(cls == 1, subn, x)
        x = np.where((cls == 2) & (inf_rank == r), (inf_sign * np.inf).astype(t), x)
        x = np.where(cls == 3, near, x)
        x = np.where(cls == 4, np.where(g.uniform(size=count) < 0.5, zeros, x), x)
        out.append(x.astype(t))
    return out


def nan_inputs(dtype, nranks, count, seed):
    """Per-rank arrays of N(0,1) values; element i of class i mod 4: 0 a NaN
    on rank 0, 1 a NaN on one later rank, 2 NaNs on two later ranks, 3 none.
    NaNs are quiet, with random sign and payload bits."""
    g = np.random.default_rng([220813707, 81, seed])
    t = np.dtype(dtype)
    ut = np.uint32 if t.itemsize == 4 else np.uint64
    mant = 23 if t.itemsize == 4 else 52
    expo = (0xFF if t.itemsize == 4 else 0x7FF) << mant
    cls = np.arange(count) % 4
    where = [np.zeros(count, bool) for _ in range(nranks)]
    r1 = g.integers(1, nranks, size=count)
    r2 = g.integers(1, nranks, size=count)
    for r in range(nranks):
        where[r] = ((cls == 0) & (r == 0)) | ((cls >= 1) & (cls <= 2) & (r1 == r)) | \
            ((cls == 2) & (r2 == r))
    out = []
    for r in range(nranks):
        x = g.standard_normal(count).astype(t)
        payload = g.integers(0, 1 << (mant - 1), size=count).astype(ut)
        sign = (g.uniform(size=count) < 0.5).astype(ut) << ut(8 * t.itemsize - 1)
        nan = (sign | ut(expo) | (ut(1) << ut(mant - 1)) | payload).view(t)
        out.append(np.where(where[r], nan, x).astype(t))
    return out


def edge_program(dtype, nranks, count, grouped=False, seed=0, inputs=edge_inputs):
    ins = inputs(dtype, nranks, count, seed)
    es = np.dtype(dtype).itemsize
    bufs, ops = [], []
    for r in range(nranks):
        b = {"in": as_bytes(ins[r])}
        rows = []
        for op in OPS:
            b["out_" + op] = np.zeros(count * es, np.uint8)
            if grouped:
                # two allreduces on the halves: one merged launch per group
                h = count // 2
                rows += [GroupStart(),
                         Allreduce("in", 0, "out_" + op, 0, h, dtype, op),
                         Allreduce("in", h * es, "out_" + op, h * es, count - h, dtype, op),
                         GroupEnd()]
            else:
                rows.append(Allreduce("in", 0, "out_" + op, 0, count, dtype, op))
        bufs.append(b)
        ops.append(rows)
    name = f"float edges {dtype} {nranks} ranks x {count}{' grouped' if grouped else ''}"
    return single_stream(nranks, bufs, ops, name=name), ins


def test_edge_inputs_hold_the_edge_values():
    """(CPU) the generator really produces signed zeros, subnormals and
    infinities, and the oracle's fold gives no NaN."""
    ins = edge_inputs("float32", 5, 600, 1)
    a = np.stack(ins)
    assert np.any(np.signbit(a) & (a == 0)) and np.any(~np.signbit(a) & (a == 0))
    sub = (a != 0) & (np.abs(a) < np.finfo(np.float32).tiny)
    assert sub.sum() > 100
    assert np.isinf(a).sum() == 100
    for op in OPS:
        assert not np.any(np.isnan(redo.fold(op, ins)))


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("nranks,count,grouped", [
    (5, 3001, False),        # fused wait-reduce kernel
    (5, 200003, False),      # split path, rank count at run time
    (16, 65539, False),      # split path, kernel unrolled over 16 ranks, ragged tail
    (6, 4099, True),         # a group's allreduces in one merged kernel
])
def test_float_edges_bit_exact(dtype, nranks, count, grouped):
    p, _ = edge_program(dtype, nranks, count, grouped)
    print(f"[gpu-case] {p.name}", file=sys.stderr, flush=True)
    ref = sim.run(p)
    g = run_program(p, stats=grouped)
    diffs = compare(p, g, ref)
    assert not diffs, "\n".join(diffs[:20])
    if grouped:
        assert g.stats.reductions_merged == 2 * len(OPS)


def test_nan_inputs_hold_nans_on_rank0_and_later_ranks():
    """(CPU) the NaN generator: quiet NaNs with payloads, on rank 0 and on
    later ranks; the oracle's MIN / MAX keep exactly rank 0's NaNs."""
    ins = nan_inputs("float32", 5, 800, 2)
    a = np.stack(ins)
    assert np.isnan(a[0]).sum() == 200 and np.isnan(a[1:]).sum() >= 400
    bits = a.view(np.uint32)[np.isnan(a)]
    assert np.all(bits & 0x00400000) and len(np.unique(bits)) > 500
    for op in ("min", "max"):
        got = redo.fold(op, ins)
        assert np.array_equal(np.isnan(got), np.isnan(a[0]))
        assert np.array_equal(got.view(np.uint32)[np.isnan(got)], a[0].view(np.uint32)[np.isnan(a[0])])
    for op in ("sum", "prod"):
        assert np.array_equal(np.isnan(redo.fold(op, ins)), np.isnan(a).any(axis=0))


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("nranks,count,grouped", [
    (5, 3001, False),        # fused wait-reduce kernel
    (5, 200003, False),      # split path, rank count at run time
    (16, 65539, False),      # split path, kernel unrolled over 16 ranks, ragged tail
    (6, 4099, True),         # a group's allreduces in one merged kernel
])
def test_nan_inputs_follow_the_reading(dtype, nranks, count, grouped):
    p, _ = edge_program(dtype, nranks, count, grouped, seed=3, inputs=nan_inputs)
    print(f"[gpu-case] NaN {p.name}", file=sys.stderr, flush=True)
    ref = sim.run(p)
    g = run_program(p)
    t = np.dtype(dtype)
    ut = np.uint32 if t.itemsize == 4 else np.uint64
    for r in range(nranks):
        for op in OPS:
            k = "out_" + op
            want = ref.buffers[r][k].view(t)
            got = g.buffers[r][k].view(t)
            if op in ("min", "max"):
                assert np.array_equal(got.view(ut), want.view(ut)), (r, op)
            else:
                wn, gn = np.isnan(want), np.isnan(got)
                assert np.array_equal(gn, wn), (r, op, np.nonzero(gn != wn)[0][:5])
                assert wn.sum() == 3 * (count // 4) + min(count % 4, 3)
                assert np.array_equal(got.view(ut)[~gn], want.view(ut)[~wn]), (r, op)
