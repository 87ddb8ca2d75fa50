"""Pins of the oracle's typemaps, pack and unpack (CPU only).

Each check compares the oracle with something fixed outside it: typemaps
worked out by hand (tests/golden), numpy slicing of the same memory, memcpy,
and a brute-force enumeration that walks the constructor tree with explicit
nested loops and no arrays.
"""
import ast
import itertools
import os

import numpy as np
import pytest

from oracle import typemap as tm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_typemaps():
    rows = []
    for line in open(os.path.join(GOLDEN, "typemaps.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tree, nums, disps = (x.strip() for x in line.split("|"))
        lb, ub, ext, size, ov = (int(v) for v in nums.split())
        rows.append((ast.literal_eval(tree), lb, ub, ext, size, bool(ov),
                     [int(v) for v in disps.split()]))
    return rows


@pytest.mark.parametrize("row", _golden_typemaps(), ids=lambda r: str(r[0]))
def test_typemap_golden(row):
    tree, lb, ub, ext, size, ov, disps = row
    t = tm.build(tree)
    assert t.disps.tolist() == disps
    assert (t.lb, t.ub, t.extent, t.size) == (lb, ub, ext, size)
    assert tm.overlaps(t, 1) == ov


def test_pack_positions_golden():
    for line in open(os.path.join(GOLDEN, "pack_counts.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tree, count, ranges = (x.strip() for x in line.split("|"))
        want = []
        for r in ranges.split():
            lo, hi = (int(v) for v in r.split("-"))
            want += list(range(lo, hi))
        got = tm.byte_positions(tm.build(ast.literal_eval(tree)), int(count)).tolist()
        assert got == want, tree


# ---------------------------------------------------------------- brute force
def _walk(tree):
    """(basic, element displacement) pairs by explicit recursion and loops;
    returns (entries, lb, ub) with lb/ub from the entries themselves."""
    size = {"uint8": 1, "int8": 1, "int32": 4, "float32": 4, "int64": 8, "float64": 8}
    if isinstance(tree, str):
        return [(tree, 0)], 0, size[tree]
    kind = tree[0]
    if kind == "contiguous":
        inner, ilb, iub = _walk(tree[2])
        shifts = [i for i in range(tree[1])]
    elif kind == "vector":
        inner, ilb, iub = _walk(tree[4])
        shifts = []
        for i in range(tree[1]):
            for j in range(tree[2]):
                shifts.append(i * tree[3] + j)
    else:
        inner, ilb, iub = _walk(tree[3])
        shifts = []
        for b, d in zip(tree[1], tree[2]):
            for j in range(b):
                shifts.append(d + j)
    ext = iub - ilb
    out = []
    for s in shifts:
        for (b, d) in inner:
            out.append((b, d + s * ext))
    if not out:
        return out, 0, 0
    lo = min(d for _, d in out)
    hi = max(d + size[b] for b, d in out)
    return out, lo, hi


def _tiny_trees():
    basics = ["int8", "int32", "float64"]
    level1 = list(basics)
    for b in basics[:2]:
        for n in range(0, 3):
            level1.append(("contiguous", n, b))
        for c, bl, st in itertools.product(range(1, 3), range(0, 3), range(1, 4)):
            level1.append(("vector", c, bl, st, b))
        level1.append(("indexed", [1, 2], [3, 0], b))
        level1.append(("indexed", [2, 0, 1], [0, 4, 9], b))
    level2 = []
    for t in level1[::3]:
        level2.append(("contiguous", 2, t))
        level2.append(("vector", 2, 2, 3, t))
        level2.append(("indexed", [1, 2], [4, 1], t))
    level3 = [("vector", 2, 1, 2, t) for t in level2[::4]]
    return level1 + level2 + level3


@pytest.mark.parametrize("tree", _tiny_trees(), ids=str)
def test_typemap_brute_force(tree):
    entries, lb, ub = _walk(tree)
    t = tm.build(tree)
    assert [d for _, d in entries] == t.disps.tolist()
    assert all(b == t.basic for b, _ in entries)
    assert (t.lb, t.ub) == (lb, ub)


# --------------------------------------------------------- library equivalents
def test_contiguous_pack_is_memcpy():
    g = np.random.default_rng(1)
    buf = g.integers(0, 256, size=4096, dtype=np.uint8)
    for off, n in [(0, 1024), (16, 7), (4, 0)]:
        got = tm.pack(buf, off, n, tm.build("int32"))
        assert got.tobytes() == buf[off: off + 4 * n].tobytes()
        got = tm.pack(buf, off, 1, tm.build(("contiguous", n, "int32")))
        assert got.tobytes() == buf[off: off + 4 * n].tobytes()


@pytest.mark.parametrize("c,bl,st", [(5, 3, 8), (2730, 3, 8), (7, 1, 2), (4, 4, 4), (3, 2, 9)])
def test_vector_pack_is_numpy_slicing(c, bl, st):
    g = np.random.default_rng(c * 100 + bl)
    a = g.standard_normal(c * st + 8).astype(np.float32)
    buf = a.view(np.uint8).copy()
    want = a[: c * st].reshape(c, st)[:, :bl].reshape(-1)
    got = tm.pack(buf, 0, 1, tm.build(("vector", c, bl, st, "float32"))).view(np.float32)
    assert np.array_equal(got, want)
    # at a column offset, as the halo exchange uses it
    want3 = a[3: 3 + c * st].reshape(c, st)[:, :bl].reshape(-1) if bl <= st - 3 else None
    if want3 is not None:
        got3 = tm.pack(buf, 12, 1, tm.build(("vector", c, bl, st, "float32"))).view(np.float32)
        assert np.array_equal(got3, want3)


def test_indexed_pack_is_concatenated_slices():
    g = np.random.default_rng(7)
    a = g.integers(-1000, 1000, size=64).astype(np.int64)
    bls, ds = [3, 1, 4, 2], [0, 5, 7, 13]
    want = np.concatenate([a[d: d + b] for b, d in zip(bls, ds)])
    got = tm.pack(a.view(np.uint8), 0, 1, tm.build(("indexed", bls, ds, "int64"))).view(np.int64)
    assert np.array_equal(got, want)


def test_vector_count_copies_is_numpy_strided():
    # count copies of vector(c, bl, st): copy k starts at k * ((c-1)*st + bl) elements
    c, bl, st, count = 4, 2, 5, 3
    ext = (c - 1) * st + bl
    a = np.arange(count * ext + 10, dtype=np.int32)
    view = np.lib.stride_tricks.as_strided(
        a, shape=(count, c, bl), strides=(ext * 4, st * 4, 4), writeable=False)
    got = tm.pack(a.view(np.uint8), 0, count, tm.build(("vector", c, bl, st, "int32")))
    assert np.array_equal(got.view(np.int32), view.reshape(-1))


# ------------------------------------------------------------------ invariants
@pytest.mark.parametrize("tree,count", [
    (("vector", 9, 3, 8, "float32"), 1),
    (("vector", 2, 2, 3, ("indexed", [2], [5], "float32")), 3),
    (("indexed", [1, 2], [3, 0], "int8"), 5),
    ("int64", 11),
])
def test_unpack_pack_identity_and_gaps(tree, count):
    t = tm.build(tree)
    n = int(tm.byte_positions(t, count).max()) + 9
    g = np.random.default_rng(3)
    src = g.integers(0, 256, size=n, dtype=np.uint8)
    sentinel = np.full(n, 0xA5, dtype=np.uint8)
    dst = sentinel.copy()
    tm.unpack(dst, 0, count, t, tm.pack(src, 0, count, t))
    pos = tm.byte_positions(t, count)
    mask = np.zeros(n, bool)
    mask[pos] = True
    assert np.array_equal(dst[mask], src[mask])          # typemap bytes carried over
    assert np.array_equal(dst[~mask], sentinel[~mask])   # gaps untouched
    assert tm.pack(dst, 0, count, t).tobytes() == tm.pack(src, 0, count, t).tobytes()


def test_truncated_unpack_writes_leading_bytes_only():
    t = tm.build(("vector", 4, 2, 3, "int32"))
    buf = np.zeros(64, np.uint8)
    data = np.arange(1, 13, dtype=np.uint8)       # 12 of 32 packed bytes
    tm.unpack(buf, 0, 1, t, data)
    assert buf[:8].tolist() == list(range(1, 9))
    assert buf[8:12].tolist() == [0] * 4           # gap
    assert buf[12:16].tolist() == [9, 10, 11, 12]
    assert not buf[16:].any()


def test_invalid_constructors():
    with pytest.raises(tm.TypeError_):
        tm.build(("vector", -1, 3, 8, "int32"))
    with pytest.raises(tm.TypeError_):
        tm.build(("indexed", [1], [-2], "int32"))
    with pytest.raises(tm.TypeError_):
        tm.build("complex64")


def test_planted_mistake_is_caught(monkeypatch):
    """A vector constructor with stride and blocklength swapped must fail the
    numpy slicing pin (the pins can see such a mistake)."""
    real = tm.vector
    monkeypatch.setattr(tm, "vector", lambda c, bl, st, t: real(c, st, bl, t))
    c, bl, st = 5, 3, 8
    a = np.arange(c * st + 8, dtype=np.float32)
    want = a[: c * st].reshape(c, st)[:, :bl].reshape(-1)
    got = tm.pack(a.view(np.uint8), 0, 1, tm.build(("vector", c, bl, st, "float32")))
    assert got.size != want.nbytes or not np.array_equal(got.view(np.float32), want)
