"""Counter-based uniform draws for branch sampling (oracle side).

The generator is SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): a 64-bit state advanced by the odd constant 0x9E3779B97F4A7C15,
whose k-th output is a fixed 64-bit finaliser applied to ``seed + k * gamma``.  A noise event
is keyed by (trajectory, layer, qubit) and takes output number
``k = 1 + (traj << 32 | layer << 16 | qubit)`` of the generator seeded with the run seed.
The uniform is the top 53 bits of that output times 2^-53, so it lies in [0, 1).

Pinned against hand-computed SplitMix64 outputs in the tests (the first outputs of seed 0
and seed 1234567 are published with the reference implementation of the generator).
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64_output(state_plus: int) -> int:
    """The SplitMix64 finaliser applied to an already-advanced state."""
    z = state_plus & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_kth(seed: int, k: int) -> int:
    """k-th output (k >= 1) of SplitMix64 started from ``seed``."""
    return splitmix64_output((seed + k * GAMMA) & MASK64)


def event_key(traj: int, layer: int, qubit: int) -> int:
    if not (0 <= traj < (1 << 31) and 0 <= layer < (1 << 16) and 0 <= qubit < (1 << 16)):
        raise ValueError("event key out of range")
    return (traj << 32) | (layer << 16) | qubit


def uniform(seed: int, traj: int, layer: int, qubit: int) -> float:
    """u in [0,1) for the noise event on ``qubit`` in ``layer`` of trajectory ``traj``."""
    out = splitmix64_kth(seed, 1 + event_key(traj, layer, qubit))
    return (out >> 11) * (1.0 / 9007199254740992.0)


def sample_branch(p, u: float) -> int:
    """Index j of the branch drawn with uniform u from weights p (Alg. 1, 'sample a
    trajectory').  Cumulative sums in order, normalised by their total; the first j with
    p_j > 0 and u < c_j is taken; if rounding leaves none, the last j with p_j > 0."""
    total = 0.0
    for x in p:
        total += float(x)
    acc = 0.0
    last = -1
    for j, x in enumerate(p):
        x = float(x)
        acc += x
        if x > 0.0:
            last = j
            if u < acc / total:
                return j
    if last < 0:
        raise ValueError("all branch weights are zero")
    return last
