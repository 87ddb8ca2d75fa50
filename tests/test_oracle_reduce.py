"""Pins of the oracle's canonical-order reductions (CPU only).

Checked against: exact Python integers reduced modulo 2^w (brute force),
closed forms, a pure-Python binary32 fold that adds in binary64 and rounds
each partial sum to binary32 (double rounding through binary64 is harmless
for one addition of two binary32 values, since 53 >= 2*24 + 2), and the
summation error bound for any order (Higham, Accuracy and Stability of
Numerical Algorithms, 2nd ed., §4.2).
"""
import struct
from fractions import Fraction

import numpy as np
import pytest

from oracle import reduce as red


def _wrap(v: int, bits: int) -> int:
    v &= (1 << bits) - 1
    return v - (1 << bits) if v >> (bits - 1) else v


def _f32(x: float) -> float:
    return struct.unpack("<f", struct.pack("<f", x))[0]


@pytest.mark.parametrize("dtype,bits", [("int32", 32), ("int64", 64)])
def test_integer_sum_is_exact_modulo(dtype, bits):
    g = np.random.default_rng(11)
    lim = 2 ** (bits - 1)
    ins = [g.integers(-lim, lim, size=257, dtype=np.int64).astype(dtype) for _ in range(16)]
    got = red.fold("sum", ins)
    for i in range(ins[0].size):
        assert int(got[i]) == _wrap(sum(int(x[i]) for x in ins), bits)


@pytest.mark.parametrize("dtype,bits", [("int32", 32), ("int64", 64)])
def test_integer_prod_is_exact_modulo(dtype, bits):
    g = np.random.default_rng(12)
    ins = [g.integers(-2**20, 2**20, size=33, dtype=np.int64).astype(dtype) for _ in range(5)]
    got = red.fold("prod", ins)
    for i in range(33):
        p = 1
        for x in ins:
            p *= int(x[i])
        assert int(got[i]) == _wrap(p, bits)


def test_sum_closed_form_base_plus_rank():
    base = np.arange(-500, 500, dtype=np.int64) * (2**35)
    ins = [base + r for r in range(16)]
    assert np.array_equal(red.fold("sum", ins), 16 * base + 120)


def test_int32_sum_wraps():
    ins = [np.array([2**31 - 1], np.int32), np.array([1], np.int32)]
    assert int(red.fold("sum", ins)[0]) == -2**31


@pytest.mark.parametrize("n", [1, 2, 3, 16, 64])
def test_float32_canonical_fold_matches_rounded_python(n):
    g = np.random.default_rng(100 + n)
    ins = [g.standard_normal(199).astype(np.float32) for _ in range(n)]
    ins[0][:3] = [1e30, -1e-30, 3.0]            # wide exponent spread
    if n > 1:
        ins[1][:3] = [-1e30, 1e-30, 2 ** -24]
    got = red.fold("sum", ins)
    for i in range(199):
        acc = float(ins[0][i])
        for r in range(1, n):
            acc = _f32(acc + float(ins[r][i]))
        assert struct.pack("<f", acc) == struct.pack("<f", float(got[i]))


def test_float32_order_matters_and_canonical_is_left_fold():
    # (1 + 2^-24) + 2^-24 in binary32: each step rounds to even -> 1.0;
    # the reverse order gives 1.0000001.
    ins = [np.array([1.0], np.float32), np.array([2**-24], np.float32),
           np.array([2**-24], np.float32)]
    assert float(red.fold("sum", ins)[0]) == 1.0
    assert float(red.fold("sum", ins[::-1])[0]) == float(np.float32(1.0) + np.float32(2**-23))


def test_float32_within_summation_bound():
    g = np.random.default_rng(5)
    n = 16
    ins = [g.standard_normal(500).astype(np.float32) for _ in range(n)]
    got = red.fold("sum", ins)
    u = 2.0 ** -24
    gamma = (n - 1) * u / (1 - (n - 1) * u)
    for i in range(500):
        exact = sum(Fraction(float(x[i])) for x in ins)
        mag = sum(abs(Fraction(float(x[i]))) for x in ins)
        assert abs(Fraction(float(got[i])) - exact) <= Fraction(gamma) * mag


def test_float64_two_inputs_is_numpy_add():
    g = np.random.default_rng(9)
    a, b = g.standard_normal(100), g.standard_normal(100)
    assert np.array_equal(red.fold("sum", [a, b]), np.add(a, b))


def test_min_max_keep_earlier_on_ties():
    ins = [np.array([0.0, 1.0], np.float32), np.array([-0.0, 1.0], np.float32)]
    mn = red.fold("min", ins)
    mx = red.fold("max", ins)
    assert not np.signbit(mn[0]) and not np.signbit(mx[0])   # +0 kept, -0 == +0
    ins = [np.array([3, -7], np.int64), np.array([-5, 9], np.int64), np.array([4, -8], np.int64)]
    assert red.fold("min", ins).tolist() == [-5, -8]
    assert red.fold("max", ins).tolist() == [4, 9]


def test_single_rank_is_identity():
    x = np.arange(10, dtype=np.float32) / 3
    assert np.array_equal(red.fold("sum", [x]), x)


def test_planted_reverse_order_is_caught(monkeypatch):
    """Folding in reverse rank order must fail the rounded-Python pin."""
    real = red.fold
    monkeypatch.setattr(red, "fold", lambda op, ins: real(op, list(ins)[::-1]))
    ins = [np.array([1.0], np.float32), np.array([2**-24], np.float32),
           np.array([2**-24], np.float32)]
    acc = 1.0
    for x in (2**-24, 2**-24):
        acc = _f32(acc + x)
    assert float(red.fold("sum", ins)[0]) != acc


def _nan32(bits):
    return np.array([bits], dtype=np.uint32).view(np.float32)[0]


@pytest.mark.parametrize("op", ["min", "max"])
def test_min_max_with_nan_keep_the_accumulator(op):
    """IEEE-754: an ordered comparison with a NaN is false.  So the fold's
    "x beats acc" never fires when either is a NaN: rank 0's NaN (payload and
    sign included) survives the fold, and a later rank's NaN is skipped."""
    qn = _nan32(0xFFC01234)                   # negative quiet NaN with a payload
    first = [np.array([qn, qn], np.float32), np.array([1.0, -5.0], np.float32),
             np.array([-2.0, 7.0], np.float32)]
    got = red.fold(op, first)
    assert got.view(np.uint32).tolist() == [0xFFC01234, 0xFFC01234]
    later = [np.array([1.0, 3.0], np.float32), np.array([qn, qn], np.float32),
             np.array([0.5, 4.0], np.float32)]
    got = red.fold(op, later)
    want = [0.5, 3.0] if op == "min" else [1.0, 4.0]
    assert got.tolist() == want and not np.any(np.isnan(got))


@pytest.mark.parametrize("op", ["sum", "prod"])
@pytest.mark.parametrize("pos", [0, 1, 2])
def test_sum_prod_with_nan_give_nan(op, pos):
    ins = [np.array([2.0, 3.0], np.float64) for _ in range(3)]
    ins[pos] = np.array([np.nan, 3.0], np.float64)
    got = red.fold(op, ins)
    assert np.isnan(got[0]) and got[1] == (9.0 if op == "sum" else 27.0)
