"""SplitMix64 counter-based generator (test infrastructure only).

Published definition: G. L. Steele, D. Lea, C. H. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014 (the SplitMix64 finaliser with
the golden-gamma increment 0x9E3779B97F4A7C15 and the multipliers
0xBF58476D1CE4E5B9, 0x94D049BB133111EB as in Vigna's public reference code).

The first output of a SplitMix64 stream whose state is ``key`` is
``mix(key + gamma)``.  The seeded perturbed start uses
key = seed XOR counter with counter = 9 * node + i, so the value of every
population is independent of any thread or loop order.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_first(keys):
    """First SplitMix64 output for each uint64 state in ``keys`` (array)."""
    z = np.asarray(keys, dtype=np.uint64) + GAMMA
    z = (z ^ (z >> np.uint64(30))) * M1
    z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def uniform01(seed, counters):
    """U in [0, 1): the top 53 bits of the output times 2^-53."""
    keys = np.uint64(seed) ^ np.asarray(counters, dtype=np.uint64)
    bits = splitmix64_first(keys) >> np.uint64(11)
    return bits.astype(np.float64) * (1.0 / 9007199254740992.0)
