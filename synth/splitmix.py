"""SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), vectorised over the draw counter.

The k-th draw (k = 0, 1, ...) of a stream seeded with ``seed`` is the finaliser
applied to ``seed + (k + 1) * 0x9E3779B97F4A7C15 (mod 2**64)``.  A uniform double in
[0, 1) is the top 53 bits of a draw times 2**-53.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_u64(seed: int, count: int) -> np.ndarray:
    """Return the first ``count`` 64-bit outputs of the stream seeded with ``seed``."""
    with np.errstate(over="ignore"):
        k = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int) -> np.ndarray:
    """``count`` doubles in [0, 1): (draw >> 11) * 2**-53."""
    z = splitmix64_u64(seed, count) >> np.uint64(11)
    return z.astype(np.float64) * (2.0 ** -53)


def uniform_pm1(seed: int, count: int) -> np.ndarray:
    """``count`` doubles in [-1, 1): 2u - 1."""
    return 2.0 * uniform01(seed, count) - 1.0


def log_uniform(seed: int, count: int, lo: float, hi: float) -> np.ndarray:
    """``count`` doubles log-uniform in [lo, hi): 10**(log10(lo) + u*(log10(hi)-log10(lo)))."""
    a, b = np.log10(lo), np.log10(hi)
    return 10.0 ** (a + uniform01(seed, count) * (b - a))
