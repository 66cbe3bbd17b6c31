"""Counter-based SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), vectorised with numpy.

The k-th output of a stream with state ``s`` is ``mix(s + (k+1)*GAMMA)``, so a
block of outputs is one vectorised call and the stream does not depend on the
numpy version's distribution algorithms.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK = (1 << 64) - 1


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def mix64_int(x: int) -> int:
    """Scalar SplitMix64 finaliser on a Python int (used to derive sub-seeds)."""
    z = x & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


class SplitMix64:
    """A SplitMix64 stream with block draws."""

    def __init__(self, seed: int):
        self.state = seed & _MASK
        self.counter = 0

    def split(self, tag: int) -> "SplitMix64":
        """Independent child stream keyed by ``tag`` (does not advance self)."""
        return SplitMix64(mix64_int(self.state ^ mix64_int((tag + 0x5151) & _MASK)))

    def u64(self, n: int) -> np.ndarray:
        k = np.arange(self.counter + 1, self.counter + 1 + n, dtype=np.uint64)
        self.counter += n
        with np.errstate(over="ignore"):
            x = np.uint64(self.state) + k * GAMMA
        return mix64(x)

    def uniform(self, n: int) -> np.ndarray:
        """Doubles in [0, 1) with 53 random bits."""
        return (self.u64(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    def uniform_open(self, n: int) -> np.ndarray:
        """Doubles in (0, 1]."""
        return 1.0 - self.uniform(n)

    def integers(self, n: int, m: int) -> np.ndarray:
        """Integers in [0, m) by multiply-shift of 32 high bits (bias < m / 2**32)."""
        hi = (self.u64(n) >> np.uint64(32)).astype(np.uint64)
        return ((hi * np.uint64(m)) >> np.uint64(32)).astype(np.int64)

    def integer(self, m: int) -> int:
        return int(self.integers(1, m)[0])

    def normal(self, n: int) -> np.ndarray:
        """Standard normals by Box-Muller (one output per pair of uniforms)."""
        u1 = self.uniform_open(n)
        u2 = self.uniform(n)
        return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)

    def geometric(self, n: int, mean: float) -> np.ndarray:
        """Geometric on {1, 2, ...} with the given mean (success prob 1/mean)."""
        p = 1.0 / mean
        if p >= 1.0:
            return np.ones(n, dtype=np.int64)
        u = self.uniform_open(n)
        return 1 + np.floor(np.log(u) / math.log(1.0 - p)).astype(np.int64)

    def permutation(self, n: int) -> np.ndarray:
        keys = self.u64(n)
        return np.argsort(keys, kind="stable").astype(np.int64)
