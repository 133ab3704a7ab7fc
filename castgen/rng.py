"""Counter-based SplitMix64 streams used by every seeded input generator.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the state advances by the odd constant
0x9E3779B97F4A7C15 and each output is the state passed through the
"mix13" finaliser.  Because output i depends only on (key, i), any element of
a stream can be drawn directly, which keeps the generators vectorised and
identical for every consumer of the inputs.

This module holds no arithmetic of the finite-element method.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    """Key of the sub-stream `stream` of seed `seed` (both non-negative ints)."""
    with np.errstate(over="ignore"):
        k = _mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + _GAMMA)
        k = _mix(k ^ np.uint64(stream & 0xFFFFFFFFFFFFFFFF))
    return np.uint64(k)


def u64(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """Outputs offset..offset+n-1 of the SplitMix64 generator keyed by (seed, stream)."""
    key = stream_key(seed, stream)
    idx = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(key + idx * _GAMMA)


def uniform(seed: int, stream: int, n: int, lo=0.0, hi=1.0, offset: int = 0) -> np.ndarray:
    """n doubles uniform on [lo, hi) from the top 53 bits of each output."""
    v = (u64(seed, stream, n, offset) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return lo + (hi - lo) * v


def permutation(seed: int, stream: int, n: int) -> np.ndarray:
    """A seeded random permutation of 0..n-1 (int64): argsort of n stream outputs."""
    keys = u64(seed, stream, n)
    return np.argsort(keys, kind="stable").astype(np.int64)
