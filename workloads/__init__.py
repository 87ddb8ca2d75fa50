"""Seeded synthetic workloads: program descriptions and their initial bytes.

This package holds no arithmetic of the method.  It only describes *what a
program asks for* (which rank posts which operation on which buffer) and draws
the initial buffer contents from seeded generators.  Both the CPU oracle and
the GPU path read these descriptions; neither imports the other.
"""
from .program import (  # noqa: F401
    Program, Send, Recv, Wait, Allreduce, User, GroupStart, GroupEnd, IN_PLACE, ANY_SOURCE,
    ANY_TAG,
    BASIC_TYPES, single_stream, as_bytes, count_messages,
)
