"""splitmix64 counter-based stream (Steele, Lea & Flood, OOPSLA 2014).

Seeded inputs for every workload are drawn from this stream so that a point
cloud is reproducible bit for bit from its seed.  The state advances by the
golden-gamma constant; each output is the state passed through the
finaliser below.  Doubles take the top 53 bits, scaled into [0, 1).
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, count):
    """Return `count` successive uint64 outputs of the stream seeded with `seed`."""
    with np.errstate(over="ignore"):
        k = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed, count):
    """`count` doubles in [0, 1) from the top 53 bits of each output."""
    return (splitmix64(seed, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform(seed, count, lo, hi):
    return lo + (hi - lo) * uniform01(seed, count)
