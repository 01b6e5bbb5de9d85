"""Counter-based generator for the initial orbitals (test infrastructure only).

The paper does not state its initial guess.  The reading adopted here: every
fragment orbital starts as uniform(-1/2, 1/2) noise drawn from SplitMix64
(G. Steele, D. Lea, C. Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), used as a counter-based generator: the k-th output
of the stream with seed s is mix(s + k * 0x9E3779B97F4A7C15) (mod 2^64), where
mix is the published finaliser.  The counter of orbital-point (alpha, i, l) is
k = ((alpha << 40) | (i << 24) | l) + 1.  A double in [0, 1) is the top 53 bits
times 2^-53.

Pins: the mix function is a bijection (checked by inverting it), the stream
reproduces the sequential SplitMix64 recurrence, and the outputs pass
uniformity checks.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64_outputs(seed: int, counters: np.ndarray) -> np.ndarray:
    """k-th SplitMix64 output for each counter k (uint64)."""
    k = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed % (1 << 64)) + k * _GOLDEN
    return _mix(state)


def splitmix64_uniform(seed: int, counters: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of each output."""
    z = splitmix64_outputs(seed, counters)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def orbital_counters(alpha: int, m: int, n: int) -> np.ndarray:
    i = np.arange(m, dtype=np.uint64)[:, None]
    l = np.arange(n, dtype=np.uint64)[None, :]
    key = (np.uint64(alpha) << np.uint64(40)) | (i << np.uint64(24)) | l
    return key + np.uint64(1)


def initial_orbitals(seed: int, alpha: int, m: int, shape) -> np.ndarray:
    """Raw (not yet orthonormal) initial orbitals of fragment alpha, (m, nz, ny, nx)."""
    n = int(np.prod(shape))
    if n >= (1 << 24) or m >= (1 << 16):
        raise ValueError("counter packing supports n < 2^24 points and m < 2^16 orbitals")
    u = splitmix64_uniform(seed, orbital_counters(alpha, m, n))
    return (u - 0.5).reshape((m,) + tuple(shape))
