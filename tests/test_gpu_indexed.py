"""Large irregular indexed messages against the oracle (§4.5: derived
datatypes are what GPU-aware libraries leave out), through the C ABI.

Irregular indexed layouts (blocks of random length at random gaps) take the
SEG map: every packed unit finds its segment either through the type's
granule table (one load) or, for elements of more than 2^22 granules, by a
binary search of the segment prefixes.  Both are run at full size, on the
per-message copy kernel and on the batch kernel (grouped), in three
directions: indexed to the same indexed type, indexed to contiguous, and
contiguous to indexed.  Receive buffers start filled with 0xEE, so a byte
written outside the typemap shows up as a difference from the oracle.

* granule table: 4,096 blocks of 1-4 float32 (gaps of 1-3), 400 copies,
  16 MiB of payload per message;
* binary search: one element of 650,000 blocks of 1, 3, .., 13 uint8 (odd
  lengths, so granules are single bytes, about 4.5 million of them: above
  the table's limit).

The oracle's result of the plain program also serves the grouped one (a
group moves the same bytes as its calls one by one, pinned in the oracle's
own tests), so the large typemaps are expanded once.
"""
import functools
import sys

import numpy as np
import pytest

from oracle import simulate as sim
from oracle import typemap as tm
from tests.gpu_runner import compare, run_program
from workloads.program import GroupEnd, GroupStart, Program, Recv, Send

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def _irregular(nblk, base, seed, maxbl, maxgap, odd=False):
    rng = np.random.default_rng([220813707, 45, seed])
    bls = rng.integers(0, (maxbl + 1) // 2, nblk) * 2 + 1 if odd else rng.integers(1, maxbl + 1, nblk)
    gaps = rng.integers(1, maxgap + 1, nblk)
    displs = np.concatenate([[0], np.cumsum(bls + gaps)[:-1]])
    return ("indexed", tuple(int(x) for x in bls), tuple(int(x) for x in displs), base)


def _program(tree, count, base, esize, grouped, seed):
    t = tm.build(tree)
    size, extent = t.size, t.extent
    n_el = size * count // esize          # basic elements of the message
    span = (count - 1) * extent + t.ub
    rng = np.random.default_rng([220813707, 46, seed])
    al = lambda x: -(-x // 256) * 256
    b0 = {"a": rng.integers(0, 256, al(span), dtype=np.uint8),
          "c": rng.integers(0, 256, al(n_el * esize), dtype=np.uint8)}
    b1 = {"x": np.full(al(span), 0xEE, np.uint8), "y": np.full(al(n_el * esize), 0xEE, np.uint8),
          "z": np.full(al(span), 0xEE, np.uint8)}
    r0 = [Send("a", 0, count, tree, 1, 0),          # indexed -> same indexed type
          Send("a", 0, count, tree, 1, 1),          # indexed -> contiguous
          Send("c", 0, n_el, base, 1, 2)]           # contiguous -> indexed
    r1 = [Recv("x", 0, count, tree, 0, 0, status="s0"),
          Recv("y", 0, n_el, base, 0, 1, status="s1"),
          Recv("z", 0, count, tree, 0, 2, status="s2")]
    if grouped:
        r0 = [GroupStart()] + r0 + [GroupEnd()]
        r1 = [GroupStart()] + r1 + [GroupEnd()]
    return Program(2, [b0, b1], [[r0], [r1]], 1,
                   name=f"indexed {len(tree[1])} blocks x {count} ({'grouped' if grouped else 'plain'})")


TABLE = dict(nblk=4096, base="float32", seed=1, maxbl=4, maxgap=3)
SEARCH = dict(nblk=650_000, base="uint8", seed=2, maxbl=13, maxgap=3, odd=True)


@functools.lru_cache(maxsize=None)
def _case(which):
    kw = TABLE if which == "table" else SEARCH
    _say(f"oracle of the {which} case ({kw['nblk']} blocks; up to a minute)")
    tree = _irregular(**kw)
    count, esize = (400, 4) if which == "table" else (1, 1)
    ref = sim.run(_program(tree, count, kw["base"], esize, False, kw["seed"]))
    assert not ref.deadlock and not any(ref.sync_errors)
    return tree, count, esize, ref


@pytest.mark.parametrize("grouped", [False, True])
def test_indexed_granule_table_full_size(grouped):
    tree, count, esize, ref = _case("table")
    p = _program(tree, count, "float32", esize, grouped, TABLE["seed"])
    _say(p.name + ": granule table, 16 MiB per message, three directions")
    diffs = compare(p, run_program(p), ref)
    assert not diffs, diffs[:5]


@pytest.mark.parametrize("grouped", [False, True])
def test_indexed_beyond_the_granule_table_full_size(grouped):
    tree, count, esize, ref = _case("search")
    assert tm.build(tree).size > 1 << 22   # more one-byte granules than a table may map
    p = _program(tree, count, "uint8", esize, grouped, SEARCH["seed"])
    _say(p.name + ": binary search (one-byte granules above the table's limit), three directions")
    diffs = compare(p, run_program(p), ref)
    assert not diffs, diffs[:5]
