"""SplitMix64 counter-based generator (Steele, Lea & Flood, OOPSLA 2014).

Value i of stream `seed` is the SplitMix64 output mix of seed + (i+1)*golden,
so any element of the stream can be produced independently of the others.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, index):
    """Raw 64-bit SplitMix64 outputs for counters `index` (uint64 array)."""
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (idx + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed, index):
    """Uniform doubles on [-1, 1) from the top 53 bits of each output."""
    z = splitmix64(seed, index)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0
