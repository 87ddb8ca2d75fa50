"""Counter-based payload generator shared (by definition, not by code) with
the serving harness kernels.

Byte j of a buffer with seed s is byte (j mod 8), little-endian, of
splitmix64(s * 2^32 + floor(j / 8)), SplitMix64 as published by Steele, Lea
and Flood ("Fast splittable pseudorandom number generators", OOPSLA 2014).
"""
import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)) & _M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
        return z ^ (z >> np.uint64(31))


def fill(seed: int, nbytes: int) -> np.ndarray:
    words = (nbytes + 7) // 8
    idx = (np.uint64(seed) << np.uint64(32)) + np.arange(words, dtype=np.uint64)
    return splitmix64(idx).astype("<u8").view(np.uint8)[:nbytes].copy()
