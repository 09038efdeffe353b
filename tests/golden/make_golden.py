"""Writes the stored expected values under tests/golden/ from the oracle only.

    python tests/golden/make_golden.py

phase_vectors.txt: (seed, r) -> SplitMix64 counter output z and
u = (z >> 11) 2^-53 of the phase reading (phi_r = 2 pi u), for a fixed set
of (seed, r) pairs including large counters and seeds near 2^64.

ensemble_ladder2x7_by0p1.txt: the exact infinite-temperature ensemble
polarisation P^ens_11(t) of Eq. (1) (exact diagonalisation, oracle.ed) for
the 14-spin ladder of Fig. 3(a): XY couplings, b_x = 1 on the legs, b_y =
b_x/10 on the rungs, site 0 polarised and observed, t = 0.05 k, k = 0..300.
ensemble_star14_dipolar.txt: the same for the dipolar star of Fig. 3(b):
M = 14, every pair coupled with b ~ N(0, 1) and a = -2b, site 0 polarised
and observed, t = 0.02 k, k = 0..250.

About three minutes of CPU each; ``python tests/golden/make_golden.py phase``
rewrites only the phase vectors.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.phase import GAMMA, MASK, _mix, phase_u  # noqa: E402
import workloads  # noqa: E402


def write_fig3a_ensemble():
    import numpy as np
    from oracle import ed
    J = workloads.ladder(7, bx=1.0, by=0.1)
    times = 0.05 * np.arange(301)
    P = ed.ensemble_P_exact(14, J, times, 0, 0)
    lines = ["# t P_ens  (Fig. 3(a) ladder 2x7, b_y/b_x = 1/10, XY, exact ensemble of Eq. (1))"]
    lines += [f"{float(t):.17g} {float(p):.17g}" for t, p in zip(times, P)]
    with open(os.path.join(HERE, "ensemble_ladder2x7_by0p1.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


def write_fig3b_ensemble():
    import numpy as np
    from oracle import ed
    J = workloads.star(14, 77, var_center=1.0, var_other=1.0, a_over_b=-2.0)
    times = 0.02 * np.arange(251)
    P = ed.ensemble_P_exact(14, J, times, 0, 0)
    lines = ["# t P_ens  (Fig. 3(b) dipolar star M=14: every pair, b ~ N(0,1) (workloads.star seed 77),"
             " a = -2b; exact ensemble of Eq. (1))"]
    lines += [f"{float(t):.17g} {float(p):.17g}" for t, p in zip(times, P)]
    with open(os.path.join(HERE, "ensemble_star14_dipolar.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


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
    if sys.argv[1:] != ["phase"]:
        write_fig3a_ensemble()
        write_fig3b_ensemble()
