"""Counter-based random numbers: SplitMix64 (Steele, Lea & Flood 2014).

``splitmix64(x)`` is the SplitMix64 output function applied to a 64-bit
counter.  A value is addressed by (seed, stream, index), so generators can
draw any element independently of array sizes or evaluation order.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    """SplitMix64 finaliser of a uint64 array (wrapping arithmetic)."""
    z = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def _key(seed, stream):
    with np.errstate(over="ignore"):
        k = splitmix64(np.uint64(seed) * np.uint64(0x100000001B3) + np.uint64(stream))
    return k


def uniform01(seed, stream, index):
    """Uniform doubles in [0, 1) for integer ``index`` (array), 53-bit resolution."""
    idx = np.asarray(index, dtype=np.int64).astype(np.uint64)
    with np.errstate(over="ignore"):
        z = splitmix64(splitmix64(idx ^ _key(seed, stream)) + _key(seed, stream))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def stream_uniform(seed, stream, n, lo=0.0, hi=1.0):
    """``n`` uniforms in [lo, hi) from one stream."""
    return lo + (hi - lo) * uniform01(seed, stream, np.arange(n, dtype=np.int64))
