"""Writes the stored expected values under tests/golden/ from the oracle only.

    python tests/golden/make_golden.py

phase_vectors.txt: (seed, r) -> SplitMix64 counter output z and
u = (z >> 11) 2^-53 of the phase reading (phi_r = 2 pi u), for a fixed set
of (seed, r) pairs including large counters and seeds near 2^64.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.phase import GAMMA, MASK, _mix, phase_u  # noqa: E402


def main():
    seeds = [0, 1, 2, 5, 33, 1000, 123456789, 2 ** 63 + 17, MASK]
    rs = [0, 1, 2, 3, 7, 100, 511, 4095, 65535, 2 ** 20 - 1, 2 ** 29 - 1, 2 ** 32 + 5, 2 ** 40 + 1]
    lines = ["# seed r z_hex u  (u = (z>>11)*2^-53, z = SplitMix64 output r+1 of stream 'seed')"]
    for s in seeds:
        for r in rs:
            z = _mix((s + (r + 1) * GAMMA) & MASK)
            lines.append(f"{s} {r} {z:016x} {phase_u(s, r)!r}")
    with open(os.path.join(HERE, "phase_vectors.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
