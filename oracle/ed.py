"""Exact ensemble results for small M (exact diagonalisation).

* ``hamiltonian_sector``: the Hamiltonian of the section "Spin systems with
  different coupling networks" written out in the Zeeman basis, restricted
  to the sector with q down spins (H is real symmetric and conserves q).
* ``ensemble_P_exact``: P^ens(t) of Eq. (1) with P = 2(W - 1/2): the
  average over the 2^(M-1) Zeeman product states with site n up (weights
  p_i = 1/2^(M-1), infinite temperature) of the polarisation of site n'
  under the exact dynamics.  Computed through the trace identity
  P^ens(t) = (4/2^M) sum_{m,l} A^n_ml A^n'_lm cos((E_m - E_l) t),
  A^s = V^T I^z_s V per sector; the tests pin it to the direct basis-state
  average (matrix exponential per basis state) at small M.
* ``ensemble_P_trotter``: the same average, Eq. (1), with the Strang
  product in place of exp(-iHt) -- the quantity a single random-phase run
  estimates (Eq. (2)), without its cross terms.
* ``phase_average_P``: Eq. (4), the mean of Eq. (2) over caller-given phase
  patterns.
* ``phase_variance_W``: the exact variance over uniform independent phases
  of W^{alpha}(t) (the Var expression after Eq. (4)),
  Var = sum_{i != i'} p_i p_i' |<Psi_i'| U^+ P_f U |Psi_i>|^2.
* ``free_fermion_P``: XY chains are exactly solvable (introduction, and item
  a) of the coupling-network section): for a chain with site 0 at one end,
  P(t) = |[g(t)]_00|^2 with g the single-particle propagator, exp(-i h t)
  for the exact dynamics or the Strang product of 2x2 bond rotations for
  the Trotterised one; ``free_fermion_profile`` gives |[g]_s0|^2 at every
  chain site s (the polarisation profile).
"""
from __future__ import annotations

import numpy as np

from .sector import sector_basis, sector_step_matrix
from .trotter import trotter_run


def hamiltonian_sector(M: int, couplings, q: int) -> np.ndarray:
    basis = sector_basis(M, q)
    d = len(basis)
    index = {int(x): k for k, x in enumerate(basis)}
    H = np.zeros((d, d))
    for (i, j, a, b) in couplings:
        m = (1 << i) | (1 << j)
        for k, x in enumerate(basis):
            x = int(x)
            bi, bj = (x >> i) & 1, (x >> j) & 1
            H[k, k] += 0.25 * a * (1.0 if bi == bj else -1.0)
            if bi != bj:
                H[index[x ^ m], k] += 0.5 * b
    return H


def _sz_diag(basis: np.ndarray, site: int) -> np.ndarray:
    return 0.5 - ((basis >> site) & 1).astype(np.float64)


def ensemble_P_exact(M: int, couplings, times, n: int, n_obs: int) -> np.ndarray:
    times = np.asarray(times, dtype=np.float64)
    P = np.zeros_like(times)
    for q in range(M + 1):
        basis = sector_basis(M, q)
        E, V = np.linalg.eigh(hamiltonian_sector(M, couplings, q))
        An = V.T @ (_sz_diag(basis, n)[:, None] * V)
        Ao = V.T @ (_sz_diag(basis, n_obs)[:, None] * V)
        W = An * Ao.T            # A^n_ml A^n'_lm
        dE = E[:, None] - E[None, :]
        for k, t in enumerate(times):
            P[k] += np.sum(W * np.cos(dE * t))
    return 4.0 * P / 2.0 ** M


def ensemble_P_trotter(M: int, couplings, dt: float, n_steps: int, n: int,
                       n_obs: int) -> np.ndarray:
    """Average of the Trotter-loop polarisation over the basis states."""
    P = np.zeros(n_steps + 1)
    for q in range(M + 1):
        basis = sector_basis(M, q)
        up_n = ((basis >> n) & 1) == 0
        if not up_n.any():
            continue
        z = 1.0 - 2.0 * ((basis >> n_obs) & 1)
        U = sector_step_matrix(M, q, couplings, dt)
        Psi = np.eye(len(basis), dtype=np.complex128)[:, up_n]
        for k in range(n_steps + 1):
            if k:
                Psi = U @ Psi
            P[k] += np.sum(z[:, None] * np.abs(Psi) ** 2)
    return P / 2.0 ** (M - 1)


def phase_average_P(M: int, couplings, dt: float, n_steps: int, n: int,
                    n_obs: int, states) -> np.ndarray:
    """Mean polarisation over a list of initial pure states, Eq. (4)."""
    acc = np.zeros(n_steps + 1)
    for psi0 in states:
        P, _, _ = trotter_run(psi0, M, couplings, dt, n_steps, n_obs)
        acc += P
    return acc / len(states)


def phase_variance_W(M: int, couplings, dt: float, k_steps, n: int,
                     n_obs: int) -> np.ndarray:
    """Exact Var_phi[W(t_k)] for independent uniform phases, each k."""
    out = []
    D = 2 ** (M - 1)
    for k in k_steps:
        tot = 0.0
        for q in range(M + 1):
            basis = sector_basis(M, q)
            up_n = ((basis >> n) & 1) == 0
            if not up_n.any():
                continue
            U = np.linalg.matrix_power(sector_step_matrix(M, q, couplings, dt), k)
            proj = (((basis >> n_obs) & 1) == 0).astype(np.float64)
            K = U.conj().T @ (proj[:, None] * U)
            Ks = K[np.ix_(up_n, up_n)]
            off = np.abs(Ks) ** 2
            tot += off.sum() - np.sum(np.diag(off))
        out.append(tot / D ** 2)
    return np.array(out)


def chain_single_particle(L: int, bonds):
    """Hopping matrix h (L x L) for chain bonds [(l, l+1, b)] : h = b/2."""
    h = np.zeros((L, L))
    for (l, m, b) in bonds:
        h[l, m] += 0.5 * b
        h[m, l] += 0.5 * b
    return h


def free_fermion_P(L: int, bonds, times=None, dt=None, n_steps=None):
    """P_00 for an XY chain with site 0 at the end.

    ``bonds`` is the ordered list of nearest-neighbour bonds (l, l+1, b) of
    the chain.  With ``times``: exact |[exp(-i h t)]_00|^2.  With ``dt`` and
    ``n_steps``: the Strang product of the bonds' 2x2 rotations, in the
    same order as the many-body factors.
    """
    if times is not None:
        w, v = np.linalg.eigh(chain_single_particle(L, bonds))
        out = []
        for t in np.asarray(times, dtype=np.float64):
            g = (v * np.exp(-1j * w * t)) @ v.T
            out.append(abs(g[0, 0]) ** 2)
        return np.array(out)
    return free_fermion_profile(L, bonds, dt, n_steps)[:, 0]


def free_fermion_profile(L: int, bonds, dt: float, n_steps: int) -> np.ndarray:
    """|[g_k]_s0|^2 for every chain site s after k Strang steps, shape
    (n_steps+1, L): the polarisation profile of an XY chain whose site 0
    starts polarised (infinite-temperature ensemble).  g_k = u^k with u the
    Strang product of the bonds' 2x2 rotations, in the many-body order."""
    tau = 0.5 * dt
    u = np.eye(L, dtype=np.complex128)
    for (l, m, b) in list(bonds) + list(bonds)[::-1]:
        t = 0.5 * b * tau
        r = np.eye(L, dtype=np.complex128)
        r[l, l] = r[m, m] = np.cos(t)
        r[l, m] = r[m, l] = -1j * np.sin(t)
        u = r @ u
    g = np.eye(L, dtype=np.complex128)
    out = [np.abs(g[:, 0]) ** 2]
    for _ in range(n_steps):
        g = u @ g
        out.append(np.abs(g[:, 0]) ** 2)
    return np.array(out)
