"""SplitMix64 counter-based generator (oracle side; test infrastructure only).

Published definition (G. Steele, D. Lea, C. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014; S. Vigna's reference
splitmix64.c): the state advances by the golden-gamma constant
0x9E3779B97F4A7C15 and each output is the state passed through the
variant-13 64-bit finalizer

    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)

Used as a counter-based generator: entry i of a stream with seed s is the
(i+1)-th output of the sequential generator started at state s, i.e.
mix(s + (i+1) * gamma).  The library implements the same definition
independently; the two share no code.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def stream(seed, n, offset=0):
    """First n outputs (uint64) of the stream with the given seed, starting at counter offset."""
    i = np.arange(offset, offset + n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed) + (i + np.uint64(1)) * GAMMA
    return mix(state)


def uniform_pm1(seed, n, offset=0):
    """Doubles in [-1, 1): 2 * (z >> 11) * 2^-53 - 1."""
    z = stream(seed, n, offset)
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


def eig_start_seed(base_seed, level, block):
    """Stream seed for the eigenvalue-estimate start vector of (level, block)."""
    with np.errstate(over="ignore"):
        return np.uint64(base_seed) + np.uint64(level) * np.uint64(0x1000003) + np.uint64(block) * np.uint64(0x10001)
