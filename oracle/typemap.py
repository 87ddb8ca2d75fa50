"""Typemaps, pack and unpack (oracle; test infrastructure only).

The paper's enqueue calls take MPI datatypes (§3.4 gives their signatures;
§4.5 contrasts them with libraries that only move contiguous intrinsic
types).  The datatype meaning is the MPI standard's, restated here:

* A datatype is a *typemap*: an ordered list of (basic type, displacement)
  pairs.  Every constructor below takes a single old type, so every typemap
  here is homogeneous and is stored as (basic name, array of displacements).
* contiguous(n, T): T's typemap repeated n times, copy i shifted by
  i * extent(T).
* vector(count, bl, stride, T): for block i < count and element j < bl, T's
  typemap shifted by (i * stride + j) * extent(T).
* indexed(count, bls, displs, T): for block i and element j < bls[i], T's
  typemap shifted by (displs[i] + j) * extent(T).
* lb = smallest displacement, ub = largest (displacement + basic size),
  extent = ub - lb, size = sum of the basic sizes.  An empty typemap has
  lb = ub = 0.
* Sending ``count`` elements of T from ``buf`` uses copy k at buf + k *
  extent(T).
* pack concatenates the bytes of every typemap entry, copy by copy and entry
  by entry, in typemap order; unpack writes successive packed bytes back to
  the same positions and touches nothing else.

All arithmetic is on plain Python ints / numpy int64 and is exact.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

BASIC_SIZE = {
    "uint8": 1, "int8": 1,
    "int32": 4, "float32": 4,
    "int64": 8, "float64": 8,
}


class TypeError_(ValueError):
    """An invalid datatype construction (reported as ERR_TYPE)."""


@dataclass(frozen=True)
class Typemap:
    basic: str
    disps: np.ndarray          # int64, in typemap order

    @property
    def esize(self) -> int:
        return BASIC_SIZE[self.basic]

    @property
    def n(self) -> int:
        return int(self.disps.size)

    @property
    def lb(self) -> int:
        return int(self.disps.min()) if self.n else 0

    @property
    def ub(self) -> int:
        return int(self.disps.max()) + self.esize if self.n else 0

    @property
    def extent(self) -> int:
        return self.ub - self.lb

    @property
    def size(self) -> int:
        return self.n * self.esize

    def signature(self):
        """Type signature: the sequence of basic types (homogeneous here)."""
        return (self.basic, self.n)


def basic(name: str) -> Typemap:
    if name not in BASIC_SIZE:
        raise TypeError_(f"unknown basic type {name!r}")
    return Typemap(name, np.zeros(1, dtype=np.int64))


def contiguous(n: int, t: Typemap) -> Typemap:
    if n < 0:
        raise TypeError_("negative count")
    shifts = np.arange(n, dtype=np.int64) * t.extent
    return Typemap(t.basic, (shifts[:, None] + t.disps[None, :]).reshape(-1))


def vector(count: int, bl: int, stride: int, t: Typemap) -> Typemap:
    if count < 0 or bl < 0 or stride < 0:
        raise TypeError_("negative count, blocklength or stride")
    i = np.arange(count, dtype=np.int64)[:, None]
    j = np.arange(bl, dtype=np.int64)[None, :]
    shifts = ((i * stride + j) * t.extent).reshape(-1)
    return Typemap(t.basic, (shifts[:, None] + t.disps[None, :]).reshape(-1))


def indexed(bls, displs, t: Typemap) -> Typemap:
    if len(bls) != len(displs):
        raise TypeError_("blocklength / displacement arrays differ in length")
    if any(b < 0 for b in bls) or any(d < 0 for d in displs):
        raise TypeError_("negative blocklength or displacement")
    parts = []
    for b, d in zip(bls, displs):
        parts.append((d + np.arange(b, dtype=np.int64)) * t.extent)
    shifts = np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)
    return Typemap(t.basic, (shifts[:, None] + t.disps[None, :]).reshape(-1))


def build(tree) -> Typemap:
    """Build a typemap from a constructor tree (see workloads.program)."""
    if isinstance(tree, str):
        return basic(tree)
    kind = tree[0]
    if kind == "contiguous":
        return contiguous(tree[1], build(tree[2]))
    if kind == "vector":
        return vector(tree[1], tree[2], tree[3], build(tree[4]))
    if kind == "indexed":
        return indexed(list(tree[1]), list(tree[2]), build(tree[3]))
    raise TypeError_(f"unknown constructor {kind!r}")


def byte_positions(t: Typemap, count: int, offset: int = 0) -> np.ndarray:
    """Byte offsets touched by ``count`` elements of t at ``offset``, in packed order."""
    copy = np.arange(count, dtype=np.int64)[:, None] * t.extent
    starts = (offset + copy + t.disps[None, :]).reshape(-1)
    return (starts[:, None] + np.arange(t.esize, dtype=np.int64)[None, :]).reshape(-1)


def overlaps(t: Typemap, count: int) -> bool:
    """True when two entries of ``count`` elements of t share a byte."""
    pos = byte_positions(t, count)
    return np.unique(pos).size != pos.size


def pack(buf: np.ndarray, offset: int, count: int, t: Typemap) -> np.ndarray:
    """The packed byte stream of ``count`` elements of t at buf[offset:]."""
    return buf[byte_positions(t, count, offset)].copy()


def unpack(buf: np.ndarray, offset: int, count: int, t: Typemap, data: np.ndarray) -> None:
    """Write the packed bytes ``data`` into buf at the positions of ``count``
    elements of t; when ``data`` is shorter than the full size only its
    leading bytes are written (a truncated or short message)."""
    pos = byte_positions(t, count, offset)
    if data.size > pos.size:
        raise ValueError("more packed bytes than the typemap holds")
    buf[pos[: data.size]] = data
