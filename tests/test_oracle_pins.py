"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here re-types the oracle's formulas: operators are rebuilt from
Kronecker products of spin-1/2 matrices and propagated with scipy's matrix
exponential, closed forms are derived by hand, brute force replaces the
oracle's shortcuts, and the phase generator is checked against the
generator's published outputs.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
from scipy import stats

import oracle
import workloads
from oracle import cref, ed, sector

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# ---------------------------------------------------------------- spin algebra
# single-site basis: index 0 = up, 1 = down (bit value 0 = up)
IZ = np.diag([0.5, -0.5])
IP = np.array([[0.0, 1.0], [0.0, 0.0]])   # |up><down|
IM = IP.T.copy()
I2 = np.eye(2)


def site_op(op, s, M):
    """Operator on site s (bit s) of M sites: kron(..., op at s, ..., ) ."""
    out = np.array([[1.0]])
    for t in range(M - 1, -1, -1):   # highest bit first in kron order
        out = np.kron(out, op if t == s else I2)
    return out


def kron_h(M, couplings):
    H = np.zeros((2 ** M, 2 ** M))
    for (i, j, a, b) in couplings:
        H += a * site_op(IZ, i, M) @ site_op(IZ, j, M)
        H += 0.5 * b * (site_op(IP, i, M) @ site_op(IM, j, M) + site_op(IM, i, M) @ site_op(IP, j, M))
    return H


def random_state(M, rng):
    v = rng.standard_normal(2 ** M) + 1j * rng.standard_normal(2 ** M)
    return v / np.linalg.norm(v)


# ------------------------------------------------------------ phase generator
def test_splitmix64_published_outputs():
    want = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_published.txt"))
            if l.strip() and not l.startswith("#")]
    s = 0
    for w in want:
        s, z = oracle.splitmix64_next(s)
        assert z == w


def test_phase_counter_is_stream_output():
    # u(seed, r) is output r+1 of the sequential stream started at `seed`
    for seed in (0, 7, 2 ** 64 - 1):
        s = seed
        for r in range(20):
            s, z = oracle.splitmix64_next(s)
            assert oracle.phase_u(seed, r) == (z >> 11) * 2.0 ** -53


def test_phase_golden_vectors_and_array_form():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "phase_vectors.txt")) if not l.startswith("#")]
    for seed, r, zhex, u in rows:
        seed, r = int(seed), int(r)
        assert oracle.phase_u(seed, r) == float(u)
        assert float(oracle.phase_u_array(seed, np.array([r]))[0]) == float(u)
        assert (int(zhex, 16) >> 11) * 2.0 ** -53 == float(u)


def test_phase_uniform():
    u = oracle.phase_u_array(12345, np.arange(200000))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / len(u))


# ------------------------------------------------------------- initial state
@pytest.mark.parametrize("M,n", [(1, 0), (4, 0), (7, 3), (9, 8)])
def test_random_phase_state_structure(M, n):
    psi = oracle.random_phase_state(M, n, seed=11)
    x = np.arange(2 ** M)
    down = ((x >> n) & 1) == 1
    assert np.all(psi[down] == 0)
    assert np.allclose(np.abs(psi[~down]) ** 2, 2.0 ** -(M - 1), rtol=1e-14, atol=0)
    assert abs(oracle.norm2(psi) - 1) < 1e-14
    assert abs(oracle.local_polarization(psi, M, n) - 1) < 1e-14
    for other in range(M):
        if other != n:   # half of the up-n configurations have `other` down
            assert abs(oracle.local_polarization(psi, M, other)) < 1e-14
    # the amplitude phase of x is 2 pi u(seed, r(x)), r = x with bit n removed
    for xx in (0, 2 ** M - 1 - (1 << n)):
        r = (xx & ((1 << n) - 1)) | ((xx >> (n + 1)) << n)
        phi = 2 * np.pi * oracle.phase_u(11, r)
        assert abs(psi[xx] * np.sqrt(2.0 ** (M - 1)) - np.exp(1j * phi)) < 1e-14


def test_product_state_has_m_minus_1_phases():
    M, n = 5, 0
    phis = np.linspace(0.3, 2.0, M)
    psi = oracle.state.product_state(M, n, phis)
    assert abs(np.linalg.norm(psi) - 1) < 1e-14
    assert abs(oracle.local_polarization(psi, M, n) - 1) < 1e-14
    # amplitude of the all-up state carries every phase
    assert abs(psi[0] - np.exp(-1j * phis[1:].sum()) / 2 ** 2) < 1e-14


# ---------------------------------------------------------------- propagator
@pytest.mark.parametrize("i,j,a,b,tau", [(0, 1, 0.0, 1.0, 0.3), (3, 1, 0.7, -1.3, 0.11),
                                         (0, 4, -2.0, 1.0, 0.05), (2, 4, 1.0, 1.0, -0.4)])
def test_factor_is_exact_two_spin_propagator(i, j, a, b, tau):
    M = 5
    rng = np.random.default_rng(1)
    psi = random_state(M, rng)
    want = sla.expm(-1j * tau * kron_h(M, [(i, j, a, b)])) @ psi
    got = psi.copy()
    oracle.apply_factor(got, M, i, j, a, b, tau)
    assert np.abs(got - want).max() < 1e-13


def test_sector_hamiltonian_matches_kronecker():
    M = 5
    J = [(0, 1, 0.3, 1.0), (1, 3, -2.0, 1.0), (2, 4, 0.0, 0.7), (0, 4, 1.1, 1.1)]
    H = kron_h(M, J)
    x = np.arange(2 ** M)
    pc = np.array([bin(v).count("1") for v in x])
    # no element couples different sectors
    assert np.abs(H[pc[:, None] != pc[None, :]]).max() == 0
    for q in range(M + 1):
        b = sector.sector_basis(M, q)
        assert np.array_equal(b, x[pc == q])
        assert np.abs(ed.hamiltonian_sector(M, J, q) - H[np.ix_(b, b)]).max() < 1e-14


def test_strang_step_is_product_of_exponentials():
    M = 5
    J = [(0, 1, 0.3, 1.0), (1, 2, 0.0, 0.8), (2, 3, -2.0, 1.0), (0, 4, 0.0, 1.5)]
    dt = 0.21
    U = np.eye(2 ** M, dtype=complex)
    for c in J + J[::-1]:
        U = sla.expm(-1j * 0.5 * dt * kron_h(M, [c])) @ U
    psi = random_state(M, np.random.default_rng(3))
    got = psi.copy()
    oracle.trotter_step(got, M, J, dt)
    assert np.abs(got - U @ psi).max() < 1e-13


def test_second_order_trotter_error():
    """|P_T - P_exact| at fixed t shrinks ~4x when dt halves."""
    M = 6
    J = workloads.ladder(3)
    psi0 = oracle.random_phase_state(M, 0, 4)
    H = kron_h(M, J)
    T = 1.6
    errs = []
    for nst in (8, 16, 32):
        P, _, _ = oracle.trotter_run(psi0, M, J, T / nst, nst, 0)
        pe = sla.expm(-1j * T * H) @ psi0
        errs.append(abs(P[-1] - oracle.local_polarization(pe, M, 0)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.0 and 3.5 < r2 < 4.5, errs


# -------------------------------------------------------------- closed forms
@pytest.mark.parametrize("M,i,j,a", [(2, 0, 1, 0.0), (2, 1, 0, 0.9), (8, 0, 7, -2.0), (6, 3, 5, 0.4)])
def test_single_bond_closed_form(M, i, j, a):
    """Only bond (n, j): P(t) = (1 + cos(b t))/2 for any seed, a and dt."""
    b, dt, n = 1.3, 0.07, i
    for seed in (1, 99):
        P, N, _ = oracle.trotter_run(oracle.random_phase_state(M, n, seed), M,
                                     [(i, j, a, b)], dt, 60, n)
        k = np.arange(61)
        assert np.abs(P - 0.5 * (1 + np.cos(b * k * dt))).max() < 1e-13
        assert np.abs(N - 1).max() < 1e-13


def test_uncoupled_observed_site_stays_polarised():
    M = 6
    J = [(1, 2, 0.0, 1.0), (2, 5, 0.5, 0.7), (3, 4, 0.0, 1.0)]
    P, _, _ = oracle.trotter_run(oracle.random_phase_state(M, 0, 2), M, J, 0.1, 30, 0)
    assert np.abs(P - 1).max() < 1e-13


def test_time_reversal_returns_initial_state():
    M = 8
    J = workloads.star(M, seed=5)
    psi0 = oracle.random_phase_state(M, 0, 6)
    _, _, psi = oracle.trotter_run(psi0, M, J, 0.03, 25, 0)
    _, _, back = oracle.trotter_run(psi, M, J, -0.03, 25, 0)
    assert np.abs(back - psi0).max() < 1e-13


def test_short_time_curvature():
    """1 - P^ens(t) = (t^2/4) sum_j b_nj^2 + O(t^4), for any a."""
    M = 6
    J = [(0, 1, 0.4, 1.0), (0, 3, -2.0, 0.6), (1, 2, 0.0, 1.2), (0, 5, 0.0, -0.3), (4, 5, 1.0, 1.0)]
    moment = sum(b * b for (i, j, a, b) in J if 0 in (i, j))
    for t in (1e-2, 5e-3):
        P = ed.ensemble_P_exact(M, J, [t], 0, 0)[0]
        assert abs((1 - P) / t ** 2 - moment / 4) < 0.05 * moment * t ** 2 * 10 + 1e-6


# ------------------------------------------------------------ ensemble (ED)
def test_exact_ensemble_equals_basis_state_average():
    """Trace identity vs Eq. (1) done literally: average over all basis
    states with site n up, each propagated with expm(-iHt)."""
    M = 6
    J = workloads.star(M, seed=1, var_center=1.0, var_other=0.3, a_over_b=-2.0)
    H = kron_h(M, J)
    times = [0.0, 0.4, 1.3, 3.0]
    for n, nobs in [(0, 0), (0, 2)]:
        got = ed.ensemble_P_exact(M, J, times, n, nobs)
        z = np.array([1 - 2 * ((x >> nobs) & 1) for x in range(2 ** M)])
        for t, g in zip(times, got):
            U = sla.expm(-1j * t * H)
            ups = [x for x in range(2 ** M) if not (x >> n) & 1]
            want = np.mean([np.sum(z * np.abs(U[:, x]) ** 2) for x in ups])
            assert abs(g - want) < 1e-12


def test_trotter_ensemble_equals_basis_state_runs():
    M = 6
    J = workloads.ladder(3)
    got = ed.ensemble_P_trotter(M, J, 0.1, 12, 0, 0)
    acc = np.zeros(13)
    for x in range(2 ** M):
        if x & 1:
            continue
        e = np.zeros(2 ** M, dtype=complex)
        e[x] = 1
        acc += oracle.trotter_run(e, M, J, 0.1, 12, 0)[0]
    assert np.abs(got - acc / 2 ** (M - 1)).max() < 1e-13


def test_fourier_pattern_identity():
    """Averaging Eq. (2) over the D phase patterns phi_r = 2 pi k r / D
    removes every cross term of Eq. (3) exactly: sum_k e^{2 pi i k(r-r')/D}
    = D delta_rr'."""
    M, n = 6, 0
    D = 2 ** (M - 1)
    J = workloads.star(M, seed=3)
    r = np.arange(D)
    states = [oracle.state.phase_pattern_state(M, n, 2 * np.pi * k * r / D) for k in range(D)]
    avg = ed.phase_average_P(M, J, 0.05, 20, n, n, states)
    ens = ed.ensemble_P_trotter(M, J, 0.05, 20, n, n)
    assert np.abs(avg - ens).max() < 1e-13


def test_exact_phase_variance_matches_empirical():
    M, n = 6, 0
    J = workloads.star(M, seed=8)
    dt, k = 0.1, 15
    var = ed.phase_variance_W(M, J, dt, [k], n, n)[0]
    nseed = 3000
    psi = np.stack([oracle.random_phase_state(M, n, s) for s in range(nseed)], axis=1).copy()
    for _ in range(k):
        for f in oracle.strang_factors(J, dt):
            oracle.apply_factor(psi, M, *f)
    W = 0.5 * (oracle.local_polarization(psi, M, n) + 1)
    emp = W.var(ddof=1)
    # sampling error of a variance: ~ var * sqrt(2/(N-1)) (kurtosis margin x2)
    assert abs(emp - var) < 4 * var * np.sqrt(2 / (nseed - 1)) * 2
    # the paper's bound Var <= max p_i = 2^-(M-1)
    assert var <= 2.0 ** -(M - 1)


def test_random_phase_deviation_shrinks_like_two_to_minus_half_M():
    """RMS_t |P^ent - P^ens| ~ 2^{-(M-1)/2} (Eq. (3) cross terms), below the
    bound std[P] <= 2 * 2^{-(M-1)/2}."""
    rms = {}
    for M in (6, 8, 10):
        J = workloads.star(M, seed=M)
        ens = ed.ensemble_P_trotter(M, J, 0.1, 40, 0, 0)
        vals = []
        for s in range(4):
            P, _, _ = oracle.trotter_run(oracle.random_phase_state(M, 0, 100 + s), M, J, 0.1, 40, 0)
            vals.append(np.sqrt(np.mean((P[1:] - ens[1:]) ** 2)))
        rms[M] = np.sqrt(np.mean(np.square(vals))) / 2.0 ** (-(M - 1) / 2)
    for M, v in rms.items():
        assert 0.1 < v < 2.0, rms


def test_free_fermion_chain():
    """XY ladder without rungs: the leg holding site 0 is an XY chain; the
    exact and the Trotterised ensembles equal |g_00|^2 of the single-particle
    propagator."""
    L = 5
    M = 2 * L
    J = workloads.ladder(L, bx=1.0, by=0.0)
    bonds = [(i, j, b) for (i, j, a, b) in J if i < L and j < L]
    Pt = ed.ensemble_P_trotter(M, J, 0.05, 150, 0, 0)
    assert np.abs(Pt - ed.free_fermion_P(L, bonds, dt=0.05, n_steps=150)).max() < 1e-12
    times = 0.05 * np.arange(151)
    Pe = ed.ensemble_P_exact(M, J, times, 0, 0)
    assert np.abs(Pe - ed.free_fermion_P(L, bonds, times=times)).max() < 1e-12
    # and 2-site chain reduces to the single-bond closed form
    assert np.abs(ed.free_fermion_P(2, [(0, 1, 1.0)], times=times) - 0.5 * (1 + np.cos(times))).max() < 1e-13


# ---------------------------------------------------------- sector restriction
def test_sector_run_equals_full_run_on_every_sector():
    M = 8
    J = workloads.ladder(4) + [(0, 5, 0.5, 0.3)]
    psi0 = oracle.random_phase_state(M, 0, 21)
    _, _, psi = oracle.trotter_run(psi0, M, J, 0.07, 9, 0)
    for q in range(M + 1):
        b = sector.sector_basis(M, q)
        v = sector.trotter_run_sector(M, q, psi0[b], J, 0.07, 9)
        assert np.abs(v - psi[b]).max() < 1e-14


def test_sector_weights_conserved():
    M = 9
    J = workloads.star(M, seed=4, a_over_b=-2.0)
    psi0 = oracle.random_phase_state(M, 0, 2)
    _, _, psi = oracle.trotter_run(psi0, M, J, 0.05, 20, 0)
    pc = np.array([bin(x).count("1") for x in range(2 ** M)])
    from math import comb
    for q in range(M + 1):
        w0 = np.sum(np.abs(psi0[pc == q]) ** 2)
        want = comb(M - 1, q) / 2 ** (M - 1)     # site 0 up: choose q downs among M-1
        assert abs(w0 - want) < 1e-14
        assert abs(np.sum(np.abs(psi[pc == q]) ** 2) - want) < 1e-13


# ------------------------------------------------------------------ C oracle
def test_c_oracle_matches_numpy_oracle():
    cref.build(force=False)
    M = 11
    J = workloads.star(M, seed=2, a_over_b=-2.0)[:30] + workloads.ladder(5)
    psi0 = oracle.random_phase_state(M, 3, 77)
    psic = cref.init_random_phase(M, 3, 77)
    assert np.abs(psic - psi0).max() < 1e-15
    P, N, psi = oracle.trotter_run(psi0, M, J, 0.04, 12, 5)
    Pc, Nc = cref.trotter_run(psic, M, J, 0.04, 12, 5)
    assert np.abs(P - Pc).max() < 1e-13 and np.abs(N - Nc).max() < 1e-13
    assert np.abs(psi - psic).max() < 1e-14


# ---------------------------------------------------------- all-site profile
def test_profile_conserves_total_polarisation_and_starts_localised():
    """Every two-spin term commutes with the total I^z, so sum_s P_s(t) is a
    constant; the random-phase state polarised at site n has P_n = 1 and
    P_s = 0 elsewhere exactly (half of its equal-weight configurations have
    site s up)."""
    M, n = 9, 4
    J = workloads.star(M, n, a_over_b=-2.0) + [(1, 7, 0.3, -0.8)]
    psi0 = oracle.random_phase_state(M, n, 5)
    Pall, N, psi = oracle.trotter_profile(psi0, M, J, 0.07, 25)
    e = np.zeros(M)
    e[n] = 1.0
    assert np.abs(Pall[0] - e).max() < 1e-13
    assert np.abs(Pall.sum(axis=1) - 1.0).max() < 1e-12
    assert np.abs(N - 1.0).max() < 1e-12
    assert np.abs(Pall[:, 2]).max() > 1e-3       # the polarisation spreads


def test_profile_free_fermion_chain_every_site():
    """Basis-state average of the profile on an XY ladder without rungs: the
    leg holding site 0 is an XY chain, so P_s = |g_s0|^2 of the single-
    particle Strang product at each of its sites, and the other leg stays at
    zero.  A wrong site index, sign or transposed propagator fails here."""
    L = 4
    M = 2 * L
    J = workloads.ladder(L, bx=1.0, by=0.0)
    bonds = [(i, j, b) for (i, j, a, b) in J if i < L and j < L]
    xs = np.arange(2 ** M)
    up0 = xs[(xs & 1) == 0]
    psi0 = np.zeros((2 ** M, len(up0)), dtype=np.complex128)
    psi0[up0, np.arange(len(up0))] = 1.0
    Pall, _, _ = oracle.trotter_profile(psi0, M, J, 0.1, 60)
    ens = Pall.mean(axis=2)
    ff = ed.free_fermion_profile(L, bonds, 0.1, 60)
    assert np.abs(ens[:, :L] - ff).max() < 1e-12
    assert np.abs(ens[:, L:]).max() < 1e-12
    assert ff[:, L - 1].max() > 0.1


def test_product_phases_are_the_counter_generator_outputs():
    """phi_l = 2 pi u(seed, l): the stored published-definition outputs of
    the generator fix the product state's phases."""
    import os
    rows = [l.split() for l in open(os.path.join(os.path.dirname(__file__), "golden", "phase_vectors.txt"))
            if not l.startswith("#")]
    for s, r, _, u in rows:
        if int(r) < 8:
            ph = oracle.product_phases(8, int(s))
            assert ph[int(r)] == 2.0 * np.pi * float(u)
    M, n = 6, 2
    ph = oracle.product_phases(M, 12)
    psi = oracle.product_state(M, n, ph)
    x = 0b101001   # sites 0, 3, 5 down; up sites other than n: 1, 4
    assert abs(psi[x] - np.exp(-1j * (ph[1] + ph[4])) / np.sqrt(2.0 ** (M - 1))) < 1e-15


def test_ladder_ensemble_light_cone():
    """Light cone of the ladder's Strang step (list order: even leg bonds, odd
    leg bonds, rungs): after k steps site 0's Heisenberg operator reaches leg
    sites 0..2k+1 only, so the infinite-temperature ensemble P of Eq. (1) at
    site 0 is the same for every 2 x L ladder with L >= 2k + 2 (a sufficient
    condition).  Checked on the oracle's Trotterised ensemble average for
    k <= 1 (L = 4, 5, 6); a ladder too short for any cone (2 x 2) already
    differs after one step, so the quantity does see the far sites.  The GPU
    tests of the brute-force ensemble at M = 16..20 rely on it for k <= 2."""
    dt = 0.05
    p4 = ed.ensemble_P_trotter(8, workloads.ladder(4), dt, 1, 0, 0)
    p5 = ed.ensemble_P_trotter(10, workloads.ladder(5), dt, 1, 0, 0)
    p6 = ed.ensemble_P_trotter(12, workloads.ladder(6), dt, 2, 0, 0)
    assert np.abs(p4 - p5).max() < 1e-14 and np.abs(p4 - p6[:2]).max() < 1e-14
    p2 = ed.ensemble_P_trotter(4, workloads.ladder(2), dt, 1, 0, 0)
    assert np.abs(p2[1] - p4[1]) > 1e-8
    assert p6[2] < 1 - 1e-3                        # the dynamics has started
