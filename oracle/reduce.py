"""Element-wise reductions in canonical rank order (oracle; test infrastructure only).

The paper says the enqueue interface extends to collectives (§3.4) without
defining a reduction order.  The reading used here: the result on every rank
is, element by element, the left fold

    out[i] = (((in_0[i] (+) in_1[i]) (+) in_2[i]) ... (+) in_{N-1}[i])

over the ranks in order 0..N-1, with (+) the MPI operation:

* integers (int32, int64): two's-complement arithmetic that wraps on
  overflow (numpy's fixed-width integer arithmetic does exactly that);
* floats (float32, float64): IEEE-754 binary arithmetic in the buffer's own
  precision, round to nearest even, one rounding per operation (numpy applies
  each elementwise operation separately, so no fused multiply-add occurs);
* min / max keep the earlier operand when the two compare equal, and also
  when either is a NaN: IEEE-754 makes every ordered comparison with a NaN
  false, so a NaN accumulator stays (its exact bits) and a NaN arriving
  later is passed over;
* sum / prod with a NaN operand give a NaN (IEEE-754); which NaN (sign and
  payload bits) is not fixed by the standard, so only "is a NaN" is
  compared there.
"""
from __future__ import annotations

import numpy as np

NP_DTYPE = {
    "int32": np.int32, "int64": np.int64,
    "float32": np.float32, "float64": np.float64,
    "uint8": np.uint8, "int8": np.int8,
}

OPS = ("sum", "prod", "min", "max")


def combine(op: str, acc: np.ndarray, x: np.ndarray) -> np.ndarray:
    """One step of the fold: acc (+) x, elementwise, in the arrays' dtype."""
    with np.errstate(over="ignore", invalid="ignore"):
        if op == "sum":
            return acc + x
        if op == "prod":
            return acc * x
        if op == "min":
            return np.where(x < acc, x, acc)
        if op == "max":
            return np.where(x > acc, x, acc)
    raise ValueError(f"unknown op {op!r}")


def fold(op: str, inputs) -> np.ndarray:
    """Left fold of the per-rank arrays ``inputs`` (rank order) under ``op``."""
    acc = np.array(inputs[0], copy=True)
    for x in inputs[1:]:
        acc = combine(op, acc, x).astype(acc.dtype, copy=False)
    return acc


def allreduce_bytes(op: str, dtype: str, count: int, inputs_bytes) -> np.ndarray:
    """Fold ``count`` elements of ``dtype`` given as per-rank byte arrays;
    returns the result as bytes."""
    t = NP_DTYPE[dtype]
    arrays = [np.frombuffer(b.tobytes(), dtype=t, count=count) for b in inputs_bytes]
    return fold(op, arrays).view(np.uint8).copy()
