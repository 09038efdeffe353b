"""Counter-based random phases for the random-phase initial state.

The paper draws the phases phi_i of the pure state at random (section
"Ensemble vs. pure entangled state", the state |Psi_pure> and its
coefficients alpha_i = sqrt(p_i) exp(i phi_i)) but names no generator.
Reading used here: phi_r = 2 pi u(seed, r) with u from SplitMix64
(G. L. Steele, D. Lea, C. H. Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), used as a counter-based generator -- u(seed, r)
is output number r+1 of the SplitMix64 stream started at state ``seed``:

    state = seed + (r + 1) * 0x9E3779B97F4A7C15          (mod 2^64)
    z = (state ^ (state >> 30)) * 0xBF58476D1CE4E5B9     (mod 2^64)
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB             (mod 2^64)
    z = z ^ (z >> 31)
    u = (z >> 11) * 2^-53                                 in [0, 1)

Pins: the first outputs of the seed-0 stream as published with the
generator's reference implementation; uniformity.
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
MASK = (1 << 64) - 1


def _mix(z: int) -> int:
    z = ((z ^ (z >> 30)) * MIX1) & MASK
    z = ((z ^ (z >> 27)) * MIX2) & MASK
    return z ^ (z >> 31)


def splitmix64_next(state: int):
    """One step of the sequential generator: returns (new_state, output)."""
    state = (state + GAMMA) & MASK
    return state, _mix(state)


def phase_u(seed: int, r: int) -> float:
    """u(seed, r) in [0, 1): output r+1 of the stream seeded with ``seed``."""
    z = _mix((seed + (r + 1) * GAMMA) & MASK)
    return (z >> 11) * 2.0 ** -53


def phase_u_array(seed: int, r: np.ndarray) -> np.ndarray:
    """Vectorised ``phase_u`` over an integer array of counters r."""
    r = np.asarray(r, dtype=np.uint64)
    with np.errstate(over="ignore"):
        s = np.uint64(seed & MASK) + (r + np.uint64(1)) * np.uint64(GAMMA)
        z = (s ^ (s >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
