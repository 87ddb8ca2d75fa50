"""CPU oracle of the MPIX-stream enqueue semantics -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously correct statement of what the
stream-ordered point-to-point and allreduce path must compute, written from
"MPIX Stream: An Explicit Solution to Hybrid MPI+X Programming" (Zhou,
Raffenetti, Guo, Thakur; EuroMPI/USA'22) and from the MPI standard's
datatype and reduction definitions that the paper builds on.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product library never does, and it shares no
code, header, table or helper with the GPU path.

Modules
  typemap   -- typemaps of derived datatypes, pack and unpack
  reduce    -- element-wise reductions in canonical rank order
  simulate  -- a deterministic single-threaded simulator of N ranks that run
               enqueue programs (matching, ordering, completion, status)

Every function is pinned by ``tests/test_oracle_*.py`` against values fixed
outside this package (closed forms, numpy slicing, hand-computed fixtures
under ``tests/golden/``, brute force on tiny inputs).  Parts with no such pin
say "parity unpinned" in their docstring.
"""
from . import typemap, reduce, simulate  # noqa: F401
