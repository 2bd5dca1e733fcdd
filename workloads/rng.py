"""Counter-based SplitMix64 (Steele, Lea, Flood 2014).

uniform(seed, k) is the k-th output (k = 0, 1, ...) of a SplitMix64 generator
whose state starts at `seed`, mapped to [0, 1) with the top 53 bits.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, k):
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (k + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed, k):
    """Uniform doubles in [0, 1) for counter values k (array-like)."""
    z = splitmix64(seed, k)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
