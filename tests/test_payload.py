"""Pins of the counter-based payload generator (CPU only)."""
import os

import numpy as np

from workloads import payload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def test_splitmix64_reference_outputs():
    want = [int(l, 16) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    gamma = np.uint64(0x9E3779B97F4A7C15)
    got = [int(payload.splitmix64(np.array([k], np.uint64) * gamma)[0]) for k in range(len(want))]
    assert got == want


def test_fill_layout():
    # byte j is byte j % 8 (little endian) of splitmix64(seed << 32 | j // 8)
    b = payload.fill(7, 21)
    w = payload.splitmix64((np.uint64(7) << np.uint64(32)) + np.arange(3, dtype=np.uint64))
    assert b.tolist() == list(w.astype("<u8").view(np.uint8)[:21])
    assert payload.fill(7, 0).size == 0
