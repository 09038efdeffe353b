"""Initial pure states (section "Testing the quantum parallelism").

``random_phase_state`` is the entangled random-phase state: the polarised
site up, every configuration r of the other M-1 sites with weight
p = 1/2^(M-1) (the infinite-temperature ensemble of the section "Spin
systems with different coupling networks") and its own phase, i.e. the
pure state sum_i alpha_i |Psi_i^m> with alpha_i = sqrt(p_i) exp(i phi_i)
of the section "Ensemble vs. pure entangled state".  The paper writes the
phase as exp(-i phi_i) for this state; with phi uniform the sign is
immaterial, and exp(+i phi) is the reading fixed for parity.

``product_state`` is the product (unentangled) state of the same section:
site n up, every other site (|down> + exp(-i phi_l) |up>)/sqrt(2).

Pins: unit norm, P[0] = 1 at the polarised site and 0 at any other site,
amplitude moduli, Fourier-pattern identity (tests).
"""
from __future__ import annotations

import numpy as np

from .phase import phase_u_array


def _r_of_x(x: np.ndarray, n: int) -> np.ndarray:
    """Index of x with bit n deleted (the ensemble member label r)."""
    x = np.asarray(x, dtype=np.uint64)
    low = x & np.uint64((1 << n) - 1)
    high = x >> np.uint64(n + 1)
    return low | (high << np.uint64(n))


def random_phase_amplitudes(M: int, n: int, seed: int, xs) -> np.ndarray:
    """Amplitudes psi0[x] for the given basis indices, computed one by one."""
    xs = np.asarray(xs, dtype=np.uint64)
    up = ((xs >> np.uint64(n)) & np.uint64(1)) == 0
    phi = 2.0 * np.pi * phase_u_array(seed, _r_of_x(xs, n))
    amp = (np.cos(phi) + 1j * np.sin(phi)) / np.sqrt(2.0 ** (M - 1))
    return np.where(up, amp, 0.0 + 0.0j)


def random_phase_state(M: int, n: int, seed: int) -> np.ndarray:
    """The full random-phase state as a complex128 vector of length 2^M."""
    return random_phase_amplitudes(M, n, seed, np.arange(2 ** M, dtype=np.uint64))


def phase_pattern_state(M: int, n: int, phases: np.ndarray) -> np.ndarray:
    """Same structure with caller-given phases phi_r (r = 0..2^(M-1)-1)."""
    x = np.arange(2 ** M, dtype=np.uint64)
    up = ((x >> np.uint64(n)) & np.uint64(1)) == 0
    r = _r_of_x(x, n).astype(np.int64)
    r = np.where(up, r, 0)
    amp = np.exp(1j * np.asarray(phases)[r]) / np.sqrt(2.0 ** (M - 1))
    return np.where(up, amp, 0.0 + 0.0j)


def product_phases(M: int, seed: int) -> np.ndarray:
    """phi_l = 2 pi u(seed, l) for l = 0..M-1: the product state's M-1 random
    phases drawn from the counter generator (the polarised site's is unused)."""
    return 2.0 * np.pi * phase_u_array(seed, np.arange(M, dtype=np.uint64))


def product_state(M: int, n: int, phis) -> np.ndarray:
    """Site n up, site l != n in (|down> + exp(-i phi_l)|up>)/sqrt(2).

    ``phis`` has one entry per site; the entry of site n is ignored.
    """
    psi = np.ones(1, dtype=np.complex128)
    for s in range(M):  # build with site s as bit s: kron puts new factor high
        if s == n:
            f = np.array([1.0, 0.0], dtype=np.complex128)
        else:
            f = np.array([np.exp(-1j * phis[s]), 1.0], dtype=np.complex128) / np.sqrt(2.0)
        psi = np.kron(f, psi)
    return psi
