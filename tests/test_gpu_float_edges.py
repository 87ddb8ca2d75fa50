"""Floating-point edge values through every reduce kernel, bit for bit.

Inputs mix, element by element: signed zeros (MIN / MAX ties between -0 and
+0 keep the earlier operand of the fold), subnormals (kept, not flushed),
+-Inf on one rank, values near the overflow threshold (sums and products
that overflow to Inf), and ordinary N(0,1) values; no element can produce a
NaN (whose payload bits are unpinned).  Every result must equal the oracle's
canonical-order fold in its bit patterns, through the fused kernel (small
reductions), the split kernel with the rank count known only at run time,
the kernel unrolled over 16 ranks, and the merged kernel of a group.
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


def edge_program(dtype, nranks, count, grouped=False, seed=0):
    ins = edge_inputs(dtype, nranks, count, seed)
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
