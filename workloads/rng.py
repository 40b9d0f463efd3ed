"""Seeded, counter-based random inputs shared by the GPU path and the oracle.

Every random number that either side consumes is produced here, from the
64-bit mixing function the paper uses to hash basis states to locales
(Section 5.1, the ``hash64_01`` listing: two xor-shift-multiply rounds and a
final xor-shift).  It is used here purely as a counter-based generator: value
number ``c`` of stream ``seed`` is ``hash64_01(seed + (c + 1) * GAMMA)`` with
GAMMA the 64-bit golden-ratio increment, which is the SplitMix64 construction.

This module holds none of the method's arithmetic (no group action, no orbit
search, no matrix elements); it only draws numbers.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def hash64_01(x: int) -> int:
    """The paper's 64-bit finalizer (Section 5.1), on a Python int."""
    x &= MASK64
    x = ((x ^ (x >> 30)) * _M1) & MASK64
    x = ((x ^ (x >> 27)) * _M2) & MASK64
    return x ^ (x >> 31)


def hash64_01_np(x: np.ndarray) -> np.ndarray:
    """Vectorised ``hash64_01`` on a uint64 array (wrapping arithmetic)."""
    x = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        x ^= x >> np.uint64(30)
        x *= np.uint64(_M1)
        x ^= x >> np.uint64(27)
        x *= np.uint64(_M2)
        x ^= x >> np.uint64(31)
    return x


def counter_u64(seed: int, counters: np.ndarray) -> np.ndarray:
    """Value ``c`` of stream ``seed``: hash64_01(seed + (c+1)*GAMMA) mod 2^64."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + (c + np.uint64(1)) * np.uint64(GAMMA)
    return hash64_01_np(z)


def u01_from_u64(u: np.ndarray) -> np.ndarray:
    """Top 53 bits as a double in [0, 1)."""
    return (np.asarray(u, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_pm1(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """x_i = 2 u_i - 1, u_i from counter (offset + i); FP64 in [-1, 1)."""
    c = np.arange(offset, offset + n, dtype=np.uint64)
    return 2.0 * u01_from_u64(counter_u64(seed, c)) - 1.0


def uniform_pm1_complex(seed: int, n: int) -> np.ndarray:
    """Complex entries: real part from counter 2i, imaginary part from 2i+1."""
    v = uniform_pm1(seed, 2 * n)
    return v[0::2] + 1j * v[1::2]


def vector(seed: int, dim: int, nrhs: int = 1, complex_: bool = False) -> np.ndarray:
    """A [dim][nrhs] row-major block of U[-1,1] entries (complex if asked).

    Entry (i, r) uses element index e = i*nrhs + r of the stream, so a
    one-column vector is the plain stream.
    """
    n = dim * nrhs
    v = uniform_pm1_complex(seed, n) if complex_ else uniform_pm1(seed, n)
    return v.reshape(dim, nrhs) if nrhs > 1 else v


def state_values(seed: int, states: np.ndarray, complex_: bool = False) -> np.ndarray:
    """A U[-1,1] value keyed by a basis *state* rather than by its index.

    Used where a vector must be known on both sides without either side
    knowing the other's index order: x[j] = f(rep_j).
    """
    s = np.asarray(states, dtype=np.uint64)
    with np.errstate(over="ignore"):
        k = hash64_01_np(s ^ np.uint64(seed & MASK64))
        if not complex_:
            return 2.0 * u01_from_u64(hash64_01_np(k)) - 1.0
        re = 2.0 * u01_from_u64(hash64_01_np(k)) - 1.0
        im = 2.0 * u01_from_u64(hash64_01_np(k ^ np.uint64(GAMMA))) - 1.0
    return re + 1j * im


def _s64(v: int) -> int:
    """A 64-bit pattern as a signed int64 value."""
    v &= MASK64
    return v - (1 << 64) if v >> 63 else v


def _hash64_01_torch(x):
    """``hash64_01`` on an int64 tensor holding 64-bit patterns (wrapping
    multiplies; logical shifts by masking the sign-extended bits)."""
    x = x ^ ((x >> 30) & ((1 << 34) - 1))
    x = x * _s64(_M1)
    x = x ^ ((x >> 27) & ((1 << 37) - 1))
    x = x * _s64(_M2)
    return x ^ ((x >> 31) & ((1 << 33) - 1))


def state_values_torch(seed: int, states):
    """``state_values`` (real) on a tensor of states stored as int64 bit
    patterns, evaluated where the tensor lives (for full-size vectors)."""
    k = _hash64_01_torch(states ^ _s64(seed))
    u = (_hash64_01_torch(k) >> 11) & ((1 << 53) - 1)
    return 2.0 * (u.double() * 2.0 ** -53) - 1.0


class Stream:
    """Sequential draws from one counter stream (for workload sampling)."""

    def __init__(self, seed: int):
        self.seed = seed
        self.c = 0

    def u64(self) -> int:
        v = hash64_01((self.seed + (self.c + 1) * GAMMA) & MASK64)
        self.c += 1
        return v

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        return lo + (hi - lo) * ((self.u64() >> 11) * 2.0 ** -53)

    def randint(self, lo: int, hi: int) -> int:
        """Integer in [lo, hi)."""
        return lo + int(self.uniform() * (hi - lo))

    def exponential(self, rate: float) -> float:
        u = self.uniform()
        return -np.log1p(-u) / rate
