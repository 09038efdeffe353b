"""Plain FP64 state-vector Trotter loop (numpy).

Follows: the Hamiltonian of the section "Spin systems with different
coupling networks" (H = sum_{i<j} a_ij I^z_i I^z_j + (b_ij/2)(I^+_i I^-_j +
I^-_i I^+_j)); the wave-function route "combined with the Trotter-Suzuki
decomposition" on vectors of size 2^M (introduction and summary); the
observable P = 2(W_11 - 1/2) of Eq. (2) and the section "Testing the quantum
parallelism", with W_11 the probability that the observed site is up.

The paper fixes no Trotter scheme.  Reading: symmetric (Strang) splitting,
one factor per coupling, list order then reverse order, each with
tau = dt/2.  Each factor is the exact two-spin propagator exp(-i tau H_ij);
in the basis (up-up, up-down, down-up, down-down) of (i, j):

    up-up, down-down:   psi -> exp(-i a tau / 4) psi
    up-down <-> down-up: exp(+i a tau / 4) [[cos t, -i sin t], [-i sin t, cos t]],
                        t = b tau / 2.

No blocking, fusion or reordering: one full pass over the vector per
factor.  Pins (tests): each factor against scipy's matrix exponential of a
Kronecker-built H_ij; the single-bond closed form; time reversal;
second-order Trotter error against the exact propagator; free fermions.
"""
from __future__ import annotations

import numpy as np


def strang_factors(couplings, dt: float):
    """One symmetric Trotter step as an ordered list of (i, j, a, b, tau)."""
    tau = 0.5 * dt
    fwd = [(int(i), int(j), float(a), float(b), tau) for (i, j, a, b) in couplings]
    return fwd + fwd[::-1]


def _pair_views(psi: np.ndarray, M: int, i: int, j: int):
    """Views of psi split by (bit_lo, bit_hi) for sites lo < hi."""
    lo, hi = (i, j) if i < j else (j, i)
    v = psi.reshape(2 ** (M - 1 - hi), 2, 2 ** (hi - lo - 1), 2, 2 ** lo, *psi.shape[1:])
    # v[:, bit_hi, :, bit_lo, :]
    return v


def apply_factor(psi: np.ndarray, M: int, i: int, j: int, a: float, b: float,
                 tau: float) -> None:
    """psi <- exp(-i tau H_ij) psi, in place (psi must be contiguous).

    ``psi`` has shape (2^M,) or (2^M, B): trailing axes are a batch of
    independent states.
    """
    if i == j:
        raise ValueError("a factor needs two distinct sites")
    v = _pair_views(psi, M, i, j)
    t = 0.5 * b * tau
    c, s = np.cos(t), np.sin(t)
    x = v[:, 1, :, 0, :].copy()   # one of the two anti-aligned configurations
    y = v[:, 0, :, 1, :].copy()   # the other one
    pa = np.exp(0.25j * a * tau)
    v[:, 1, :, 0, :] = pa * (c * x - 1j * s * y)
    v[:, 0, :, 1, :] = pa * (-1j * s * x + c * y)
    if a != 0.0:
        pd = np.exp(-0.25j * a * tau)
        v[:, 0, :, 0, :] *= pd
        v[:, 1, :, 1, :] *= pd


def trotter_step(psi: np.ndarray, M: int, couplings, dt: float) -> None:
    for (i, j, a, b, tau) in strang_factors(couplings, dt):
        apply_factor(psi, M, i, j, a, b, tau)


def local_polarization(psi: np.ndarray, M: int, site: int):
    """sum_x (1 - 2 bit_site(x)) |psi_x|^2 = 2 W - (norm), W = P(site up).

    Returns a float, or an array over the trailing batch axes of ``psi``.
    """
    p = (psi.real ** 2 + psi.imag ** 2).reshape(2 ** (M - 1 - site), 2, 2 ** site,
                                                 *psi.shape[1:])
    out = p[:, 0, :].sum(axis=(0, 1)) - p[:, 1, :].sum(axis=(0, 1))
    return float(out) if psi.ndim == 1 else out


def norm2(psi: np.ndarray):
    out = (psi.real ** 2 + psi.imag ** 2).sum(axis=0)
    return float(out) if psi.ndim == 1 else out


def trotter_profile(psi0: np.ndarray, M: int, couplings, dt: float, n_steps: int):
    """As ``trotter_run``, with the observable of Eq. (2) read at every site.

    Returns (Pall, N, psi): Pall[k, s] is the polarisation of site s after k
    steps (shape (n_steps+1, M) plus any batch axes of psi0), N[k] the norm.
    Pins (tests): the total polarisation sum_s Pall[k, s] is conserved (every
    two-spin term commutes with the total I^z); the basis-state average on an
    XY chain equals |g_s0|^2 of the single-particle Strang product at every
    site s.
    """
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    Pall = np.empty((n_steps + 1, M) + psi.shape[1:])
    N = np.empty((n_steps + 1,) + psi.shape[1:])

    def observe(k):
        for s in range(M):
            Pall[k, s] = local_polarization(psi, M, s)
        N[k] = norm2(psi)

    observe(0)
    for k in range(1, n_steps + 1):
        trotter_step(psi, M, couplings, dt)
        observe(k)
    return Pall, N, psi


def trotter_run(psi0: np.ndarray, M: int, couplings, dt: float, n_steps: int,
                observed: int):
    """Evolve a copy of psi0 for n_steps Strang steps.

    Returns (P, N, psi) with P[k], N[k] after k steps (k = 0..n_steps).
    """
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    P = np.empty(n_steps + 1)
    N = np.empty(n_steps + 1)
    P[0] = local_polarization(psi, M, observed)
    N[0] = norm2(psi)
    for k in range(1, n_steps + 1):
        trotter_step(psi, M, couplings, dt)
        P[k] = local_polarization(psi, M, observed)
        N[k] = norm2(psi)
    return P, N, psi
