"""Host logic of the datatype compiler against the oracle's typemaps (CPU only).

Type construction and the size / extent queries run on the host; they are
checked against the oracle for every tree of the typemap pins."""
import os

import pytest

from oracle import typemap as tm
from tests.test_oracle_typemap import _golden_typemaps, _tiny_trees

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2208_13707_amd", "libmpixs.so")


def _build(M, tree):
    if isinstance(tree, str):
        return 0, M.BASIC[tree]
    if tree[0] == "contiguous":
        rc, t = _build(M, tree[2])
        return M.mpixs_type_contiguous(tree[1], t) if rc == 0 else (rc, 0)
    if tree[0] == "vector":
        rc, t = _build(M, tree[4])
        return M.mpixs_type_vector(tree[1], tree[2], tree[3], t) if rc == 0 else (rc, 0)
    rc, t = _build(M, tree[3])
    return M.mpixs_type_indexed(list(tree[1]), list(tree[2]), t) if rc == 0 else (rc, 0)


TREES = [r[0] for r in _golden_typemaps()] + _tiny_trees() + [
    ("vector", 43690, 3, 8, "float32"),
    ("vector", 1000000, 2, 2, "int64"),
    ("indexed", [3, 3, 3], [0, 8, 16], "float32"),
    ("contiguous", 3, ("indexed", [2], [5], "float32")),
]


@pytest.mark.parametrize("tree", TREES, ids=str)
def test_size_and_extent_match_oracle(tree):
    if not os.path.exists(LIB):
        pytest.fail("libmpixs.so is not built")
    from paper_2208_13707_amd import mpixs as M
    rc, t = _build(M, tree)
    assert rc == 0
    want = tm.build(tree)
    assert M.mpixs_type_size(t) == (0, want.size)
    assert M.mpixs_type_get_extent(t) == (0, want.lb, want.extent)


def test_invalid_constructors_are_rejected():
    from paper_2208_13707_amd import mpixs as M
    assert M.mpixs_type_vector(-1, 3, 8, M.FLOAT32)[0] == 2       # ERR_COUNT
    assert M.mpixs_type_vector(2, 3, -8, M.FLOAT32)[0] == 3       # ERR_TYPE
    assert M.mpixs_type_indexed([1], [-2], M.INT32)[0] == 3
    assert M.mpixs_type_contiguous(2, 12345)[0] == 3
