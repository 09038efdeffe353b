"""Trotter loop restricted to one sector of fixed total S^z.

Every term of the paper's Hamiltonian (section "Spin systems with different
coupling networks": I^z_i I^z_j and the flip-flop I^+_i I^-_j + h.c.)
conserves the number of down spins q = popcount(x), so each two-spin factor
maps the sector {x : popcount(x) = q} onto itself.  Running the same
Strang product (same factor definition and order as ``trotter.py``) on the
sector's amplitudes alone gives exactly the full run's amplitudes there.
This lets the oracle produce element-by-element expected amplitudes for
states far too large to hold (q <= 3 or q >= M-3 at M = 30 has at most a
few thousand entries).

Pins (tests): equality with the full Trotter loop on every sector at small
M; sector weights conserved.
"""
from __future__ import annotations

from functools import lru_cache
from itertools import combinations

import numpy as np


@lru_cache(maxsize=64)
def sector_basis(M: int, q: int) -> np.ndarray:
    """Sorted basis indices x in [0, 2^M) with exactly q set bits."""
    xs = [sum(1 << b for b in c) for c in combinations(range(M), q)]
    return np.array(sorted(xs), dtype=np.int64)


def _pair_positions(basis: np.ndarray, i: int, j: int):
    bi = (basis >> i) & 1
    bj = (basis >> j) & 1
    sel = np.nonzero((bi == 0) & (bj == 1))[0]
    partner = basis[sel] ^ ((1 << i) | (1 << j))
    pos = np.searchsorted(basis, partner)
    same = np.nonzero(bi == bj)[0]
    return sel, pos, same


def apply_factor_sector(vec: np.ndarray, basis: np.ndarray, i: int, j: int,
                        a: float, b: float, tau: float, _cache={}) -> None:
    """exp(-i tau H_ij) on the sector amplitudes ``vec`` (in place).

    Same matrix as ``trotter.apply_factor``: on the anti-aligned pair
    (bit_i = 0, bit_j = 1) <-> (1, 0): exp(+i a tau/4) [[c, -i s], [-i s, c]]
    with c, s = cos, sin(b tau / 2); aligned configurations get
    exp(-i a tau / 4).
    """
    key = (id(basis), len(basis), i, j)
    if key not in _cache:
        _cache[key] = _pair_positions(basis, i, j)
    sel, pos, same = _cache[key]
    t = 0.5 * b * tau
    c, s = np.cos(t), np.sin(t)
    pa = np.exp(0.25j * a * tau)
    x = vec[sel].copy()
    y = vec[pos].copy()
    vec[sel] = pa * (c * x - 1j * s * y)
    vec[pos] = pa * (-1j * s * x + c * y)
    if a != 0.0:
        vec[same] *= np.exp(-0.25j * a * tau)


def trotter_run_sector(M: int, q: int, vec0: np.ndarray, couplings, dt: float,
                       n_steps: int, record_every: int = 0):
    """Evolve the sector-q amplitudes ``vec0`` (ordered as ``sector_basis``).

    Returns the final amplitudes, and if ``record_every`` > 0 also a dict
    {k: amplitudes after k steps} for k = record_every, 2*record_every, ...
    """
    basis = sector_basis(M, q)
    vec = np.array(vec0, dtype=np.complex128, copy=True)
    tau = 0.5 * dt
    seq = [(int(i), int(j), float(a), float(b)) for (i, j, a, b) in couplings]
    seq = seq + seq[::-1]
    rec = {}
    for k in range(1, n_steps + 1):
        for (i, j, a, b) in seq:
            apply_factor_sector(vec, basis, i, j, a, b, tau)
        if record_every and k % record_every == 0:
            rec[k] = vec.copy()
    return (vec, rec) if record_every else vec


def sector_step_matrix(M: int, q: int, couplings, dt: float) -> np.ndarray:
    """Matrix of one Strang step restricted to sector q (columns = images)."""
    basis = sector_basis(M, q)
    d = len(basis)
    U = np.eye(d, dtype=np.complex128)
    tau = 0.5 * dt
    seq = [(int(i), int(j), float(a), float(b)) for (i, j, a, b) in couplings]
    seq = seq + seq[::-1]
    for (i, j, a, b) in seq:
        apply_factor_sector(U, basis, i, j, a, b, tau)
    return U
