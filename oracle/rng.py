"""Counter-based SplitMix64 stream (oracle's own implementation).

Test infrastructure only.

SplitMix64 as published by Steele, Lea and Flood, "Fast splittable
pseudorandom number generators" (OOPSLA 2014): the i-th output of a stream
with seed s is mix64(s + (i + 1) * 0x9E3779B97F4A7C15) with the variant-13
finaliser.  Used for the power-iteration start vector, whose distribution the
paper does not fix (reading: uniform on [-1, 1)).
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, n):
    with np.errstate(over="ignore"):
        i = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed, n):
    """Doubles in [-1, 1): 53 high bits of each output scaled by 2^-52, minus 1."""
    z = splitmix64(seed, n)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0
