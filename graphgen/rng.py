"""Counter-based SplitMix64 streams, vectorised with numpy.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the generator's state advances by the odd constant
GAMMA and each output is the state passed through a fixed 64-bit mixing
function.  Output i of the stream seeded with ``seed`` is therefore
``mix(seed + (i + 1) * GAMMA)``, which lets a whole block of outputs be drawn
at once with no sequential dependence.

Bounded integers use Lemire's multiply-and-reject method ("Fast random integer
generation in an interval", ACM TOMACS 2019); doubles in [0, 1) take the top 53
bits.  Everything here is input generation only: none of it computes any part of
betweenness centrality.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1

# Base seed of every workload; workload c uses BASE_SEED + c.
BASE_SEED = 0x0809190600


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied elementwise to a uint64 array."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _mix64_int(z: int) -> int:
    z &= _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def substream(seed: int, *keys: int) -> int:
    """Derive an independent stream seed from ``seed`` and integer keys."""
    s = seed & _MASK64
    for k in keys:
        s = _mix64_int((s + ((int(k) + 1) * 0x9E3779B97F4A7C15)) & _MASK64)
    return s


class Stream:
    """One SplitMix64 stream; draws advance an internal counter."""

    def __init__(self, seed: int):
        self.seed = int(seed) & _MASK64
        self.counter = 0

    def u64(self, count: int) -> np.ndarray:
        idx = np.arange(self.counter + 1, self.counter + 1 + count, dtype=np.uint64)
        self.counter += count
        with np.errstate(over="ignore"):
            return mix64(np.uint64(self.seed) + idx * GAMMA)

    def doubles(self, count: int) -> np.ndarray:
        """Uniform doubles in [0, 1): (x >> 11) * 2^-53."""
        return (self.u64(count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def bounded(self, bounds) -> np.ndarray:
        """Uniform integers in [0, r) for each r in ``bounds`` (0 < r < 2^32).

        Lemire's method: the high 64 bits of x*r are the draw; a draw whose low
        64 bits fall below (2^64 - r) mod r is rejected and redrawn.
        """
        r = np.asarray(bounds, dtype=np.uint64).ravel()
        if r.size == 0:
            return np.zeros(0, dtype=np.int64)
        if np.any(r == 0) or np.any(r >= np.uint64(1 << 32)):
            raise ValueError("bounds must lie in [1, 2^32)")
        out = np.empty(r.size, dtype=np.uint64)
        todo = np.arange(r.size)
        while todo.size:
            x = self.u64(todo.size)
            rr = r[todo]
            with np.errstate(over="ignore"):
                x_hi = x >> np.uint64(32)
                x_lo = x & np.uint64(0xFFFFFFFF)
                lo_prod = x_lo * rr
                hi = (x_hi * rr + (lo_prod >> np.uint64(32))) >> np.uint64(32)
                low64 = x * rr
                thresh = (np.uint64(0) - rr) % rr
            ok = low64 >= thresh
            out[todo[ok]] = hi[ok]
            todo = todo[~ok]
        return out.astype(np.int64)

    def permutation(self, n: int) -> np.ndarray:
        """Uniform random permutation of range(n): sort by random 64-bit keys."""
        keys = self.u64(n)
        return np.argsort(keys, kind="stable").astype(np.int64)
