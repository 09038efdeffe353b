"""Parity at the full problem sizes over long runs, in the launch
configuration the benchmark times (default tile shape, long runs on the
repeating plan).

The oracle's full loop compares every amplitude of the M = 28-30 states on
a step prefix (test_gpu_fullsize_oracle.py); over runs of hundreds of
steps, where that loop would take hours:
* amplitudes of the low and high total-S^z sectors (every factor conserves
  the number of down spins) are computed by the oracle's sector-restricted
  Trotter loop and compared element by element;
* the observable is checked against closed forms that hold at any size
  (single bond; XY chain = free fermions, with the rungs present at b = 0 so
  that the plan is the benchmark's);
* time reversal returns the initial amplitudes, which the oracle computes
  one by one;
* the FP32 path is compared with the FP64 path over the whole run.
For the 2 x 12 ladder (M = 24) the oracle's full loop runs on a prefix.
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle import cref, ed, sector
import paper_0710_3747_amd as spq
from gpu_helpers import TOL_P, gpu_evolve, note

pytestmark = pytest.mark.gpu
C64, C128 = spq.SPIN_C64, spq.SPIN_C128
PRECS = [C128, C64]


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    spq.load_library()
    cref.build(force=False)
    yield
    torch.cuda.empty_cache()


def sector_check(psi_t, M, J, dt, steps, seed, prec, sectors):
    """GPU amplitudes vs the sector-restricted oracle loop on `sectors`."""
    import torch
    scale = 2.0 ** (-(M - 1) / 2)          # modulus of every initial amplitude
    tol = 1e-10 if prec == C128 else 2e-4
    for q in sectors:
        basis = sector.sector_basis(M, q)
        v0 = oracle.random_phase_amplitudes(M, 0, seed, basis.astype(np.uint64))
        want = sector.trotter_run_sector(M, q, v0, J, dt, steps)
        idx = torch.from_numpy(basis).to(psi_t.device)
        got = psi_t[idx].cpu().numpy().astype(np.complex128)
        err = np.abs(got - want).max() / scale
        assert err < tol, f"sector {q}: rel err {err:.3e}"


def free_mem_gib():
    import torch
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    return free / 2 ** 30


@pytest.mark.parametrize("prec", PRECS)
def test_ladder_2x12_prefix_matches_full_oracle(prec):
    """2 x 12 ladder (M = 24): the oracle's full loop on a 6-step prefix."""
    M, J, dt = 24, workloads.ladder(12), 0.05
    note("ladder 2x12 prefix", prec)
    P, N, psi, _ = gpu_evolve(prec, M, J, dt, 6, 0, seed=2)
    psiw = np.ascontiguousarray(oracle.random_phase_state(M, 0, 2))
    Pw, Nw = cref.trotter_run(psiw, M, J, dt, 6, 0)
    assert np.abs(P - Pw).max() < TOL_P[prec]
    err = np.abs(psi - psiw).max() / np.abs(psiw).max()
    assert err < (1e-10 if prec == C128 else 1e-4)


def test_ladder_2x12_full_run_fp32_vs_fp64_and_sectors():
    """2 x 12 ladder, dt = 0.05, 2000 steps: complex64 with FP64 reductions
    against complex128, P within 1e-4 at every step; low sectors against the
    oracle after the full run."""
    M, J, dt, steps = 24, workloads.ladder(12), 0.05, 2000
    note("ladder 2x12 2000 steps")
    P64, N64, _, t64 = gpu_evolve(C128, M, J, dt, steps, 0, seed=2, keep_state=False)
    sector_check(t64, M, J, dt, steps, 2, C128, [0, 1, 2, 22, 23, 24])
    del t64
    P32, N32, _, t32 = gpu_evolve(C64, M, J, dt, steps, 0, seed=2, keep_state=False)
    sector_check(t32, M, J, dt, steps, 2, C64, [1, 2])
    assert np.abs(P32 - P64).max() < 1e-4
    assert np.abs(N64 - 1).max() < 1e-10 and np.abs(N32 - 1).max() < 1e-4


# the default shape, then the complex64 shapes the autotuner chooses between
# for the benchmark (tile bits, register bits, coalescing bits)
LADDER_SHAPES = [(C128, None), (C64, None), (C64, (14, 5, 6)), (C64, (14, 4, 4)), (C64, (14, 5, 5))]


@pytest.mark.parametrize("prec,shape", LADDER_SHAPES, ids=[("c64" if p == C64 else "c128") + ("-default" if s is None else "-k%d-r%d-c%d" % s)
                              for p, s in LADDER_SHAPES])
def test_ladder_2x15_sectors_periodic_plan(prec, shape):
    """2 x 15 ladder (M = 30, 8 / 16 GiB), 100 steps: long enough for the
    repeating plan the benchmark uses; sectors with <= 2 or >= 28 spins down
    against the oracle."""
    M, J, dt, steps = 30, workloads.ladder(15), 0.05, 100
    opts = None if shape is None else dict(zip(("tile_bits", "reg_bits", "coalesce_bits"), shape))
    info = spq.spin_describe_plan(prec, M, J, dt, steps, 0, None if opts is None else spq.Options(**opts))
    assert info["path"] == 2 and info["period_steps"] > 0
    note("ladder 2x15 sectors", prec, shape)
    P, N, _, t = gpu_evolve(prec, M, J, dt, steps, 0, seed=5, opts=opts, keep_state=False)
    sector_check(t, M, J, dt, steps, 5, prec, [0, 1, 2, 28, 29])
    assert abs(P[0] - 1) < TOL_P[prec]
    assert np.abs(N - 1).max() < (1e-10 if prec == C128 else 1e-4)


@pytest.mark.parametrize("prec", PRECS)
def test_ladder_2x15_free_fermion_closed_form(prec):
    """Rungs at b = 0 (same plan as the full ladder): site 0's leg is an XY
    chain, whose ensemble P is |g_00|^2 of the Trotterised single-particle
    propagator; one random-phase state deviates from it by O(2^{-(M-1)/2})
    (Eq. (3) cross terms; variance bound after Eq. (4))."""
    L, dt, steps = 15, 0.05, 300
    M = 2 * L
    J = workloads.ladder(L, bx=1.0, by=0.0)
    note("free fermion M=30", prec)
    P, _, _, _ = gpu_evolve(prec, M, J, dt, steps, 0, seed=5, keep_state=False)
    bonds = [(i, j, b) for (i, j, a, b) in J if i < L and j < L]
    want = ed.free_fermion_P(L, bonds, dt=dt, n_steps=steps)
    dev = np.abs(P - want)
    sigma = 2.0 ** (-(M - 1) / 2)
    assert dev.max() < 12 * sigma, dev.max() / sigma
    assert np.sqrt(np.mean(dev ** 2)) < 3 * sigma


@pytest.mark.parametrize("prec", PRECS)
def test_single_bond_top_bits_M30(prec):
    """Only bond (0, 29) at M = 30: P = (1 + cos(b t))/2 exactly."""
    M, b, dt, steps = 30, 1.3, 0.05, 40
    note("single bond M=30", prec)
    P, N, _, _ = gpu_evolve(prec, M, [(0, 29, 0.0, b)], dt, steps, 0, seed=9, keep_state=False)
    k = np.arange(steps + 1)
    assert np.abs(P - 0.5 * (1 + np.cos(b * k * dt))).max() < TOL_P[prec]


def test_time_reversal_echo_M30():
    """30 steps at dt then 30 at -dt return the initial state; sampled
    amplitudes against the oracle's initial state computed one by one."""
    import torch
    M, J, dt = 30, workloads.ladder(15), 0.05
    note("echo M=30")
    _, _, _, t = gpu_evolve(C128, M, J, dt, 30, 0, seed=5, keep_state=False)
    _, _, _, t = gpu_evolve(C128, M, J, -dt, 30, 0, psi=t, keep_state=False)
    rng = np.random.default_rng(1)
    xs = np.unique(rng.integers(0, 2 ** M, size=20000))
    got = t[torch.from_numpy(xs).cuda()].cpu().numpy()
    want = oracle.random_phase_amplitudes(M, 0, 5, xs.astype(np.uint64))
    assert np.abs(got - want).max() < 1e-11


@pytest.mark.parametrize("prec", PRECS)
def test_star_28_sectors(prec):
    """Star M = 28 (378 couplings, J_0j ~ N(0,1), J_ij ~ N(0, 0.1), in the
    workload's block order), dt = 0.02: sectors with <= 2 spins down after
    12 steps."""
    cfg = workloads.STAR_M28
    M = cfg["M"]
    J = workloads.star_m28()
    note("star 28", prec)
    P, N, _, t = gpu_evolve(prec, M, J, cfg["dt"], 12, 0, seed=cfg["seed"], keep_state=False)
    sector_check(t, M, J, cfg["dt"], 12, cfg["seed"], prec, [0, 1, 2, 27])
    assert np.abs(N - 1).max() < (1e-10 if prec == C128 else 1e-4)


def test_fp32_vs_fp64_ladder_2x15():
    M, J, dt, steps = 30, workloads.ladder(15), 0.05, 200
    note("fp32 vs fp64 M=30")
    P64, _, _, _ = gpu_evolve(C128, M, J, dt, steps, 0, seed=5, keep_state=False)
    P32, _, _, _ = gpu_evolve(C64, M, J, dt, steps, 0, seed=5, keep_state=False)
    assert np.abs(P32 - P64).max() < 1e-4


@pytest.mark.parametrize("prec,M", [(C64, 34), (C128, 33)])
def test_maximum_sizes_single_bond(prec, M):
    """The largest states the ABI accepts (128 GiB): closed form."""
    if free_mem_gib() < 130:
        pytest.skip("not enough device memory for a 128 GiB state")
    b, dt, steps = 0.9, 0.1, 6
    note("max size", prec, M)
    P, N, _, _ = gpu_evolve(prec, M, [(0, M - 1, 0.2, b)], dt, steps, 0, seed=1, keep_state=False)
    k = np.arange(steps + 1)
    assert np.abs(P - 0.5 * (1 + np.cos(b * k * dt))).max() < TOL_P[prec]
    assert np.abs(N - 1).max() < (1e-10 if prec == C128 else 1e-4)


@pytest.mark.parametrize("prec,M", [(C64, 34), (C128, 33)])
def test_maximum_sizes_profile_single_bond(prec, M):
    """All-site profile at the largest states: the bond's two sites follow
    (1 +- cos bt)/2, every other site stays at zero, the norm at one."""
    import torch
    if free_mem_gib() < 130:
        pytest.skip("not enough device memory for a 128 GiB state")
    from gpu_helpers import gpu_profile
    b, dt, steps = 0.9, 0.1, 4
    note("max size profile", prec, M)
    Pall, N, _ = gpu_profile(prec, M, [(0, M - 1, 0.2, b)], dt, steps, 0, 1, keep_state=False)
    c = np.cos(b * np.arange(steps + 1) * dt)
    tol = TOL_P[prec]
    assert np.abs(Pall[:, 0] - 0.5 * (1 + c)).max() < tol
    assert np.abs(Pall[:, M - 1] - 0.5 * (1 - c)).max() < tol
    assert np.abs(Pall[:, 1:M - 1]).max() < tol
    assert np.abs(N - 1).max() < (1e-10 if prec == C128 else 1e-4)
    torch.cuda.empty_cache()


def test_mfma_engine_ladder_2x15_sectors_and_vs_butterflies():
    """Matrix engine at M = 30 (8 GiB complex64): sectors with <= 2 spins
    down against the oracle, and P against the butterfly path."""
    M, J, dt, steps = 30, workloads.ladder(15), 0.05, 20
    note("mfma engine M=30")
    P1, N1, _, t = gpu_evolve(C64, M, J, dt, steps, 0, seed=5, opts={"engine": 1}, keep_state=False)
    sector_check(t, M, J, dt, steps, 5, C64, [0, 1, 2])
    del t
    P0, _, _, _ = gpu_evolve(C64, M, J, dt, steps, 0, seed=5, keep_state=False)
    assert np.abs(P1 - P0).max() < 1e-5
    assert np.abs(N1 - 1).max() < 1e-4


@pytest.mark.parametrize("prec", PRECS)
def test_profile_ladder_2x15_free_fermions_every_site(prec):
    """All-site profile at M = 30 on the benchmark's plan shape (rungs at
    b = 0): the sites of site 0's leg follow |g_s0|^2 of the Trotterised
    single-particle propagator within the random-phase deviation, the other
    leg stays at zero within it, the total polarisation is conserved, and the
    last row equals spin_local_polarization of the final state."""
    import torch
    from gpu_helpers import gpu_profile
    L, dt, steps = 15, 0.05, 100
    M = 2 * L
    J = workloads.ladder(L, bx=1.0, by=0.0)
    note("profile free fermion M=30", prec)
    Pall, N, _ = gpu_profile(prec, M, J, dt, steps, 0, 5, keep_state=False)
    bonds = [(i, j, b) for (i, j, a, b) in J if i < L and j < L]
    want = ed.free_fermion_profile(L, bonds, dt, steps)
    sigma = 2.0 ** (-(M - 1) / 2)
    assert np.abs(Pall[:, :L] - want).max() < 12 * sigma
    assert np.abs(Pall[:, L:]).max() < 12 * sigma
    tol = 1e-10 if prec == C128 else 1e-4
    assert np.abs(Pall.sum(axis=1) - 1.0).max() < tol
    assert np.abs(N - 1.0).max() < tol
    torch.cuda.empty_cache()


def test_profile_last_row_is_final_state_M30():
    import torch
    M, dt, steps = 30, 0.05, 7
    J = workloads.ladder(15)
    note("profile last row M=30")
    psi = torch.empty(2 ** M, dtype=torch.complex64, device="cuda")
    spq.spin_init_random_phase(psi, M, 0, 9)
    Pall = torch.zeros((steps + 1) * M, dtype=torch.float64, device="cuda")
    spq.spin_trotter_evolve_profile(psi, M, J, dt, steps, Pall, None)
    out = torch.zeros(M, dtype=torch.float64, device="cuda")
    for s in range(M):
        spq.spin_local_polarization(psi, M, s, out[s:s + 1])
    torch.cuda.synchronize()
    last = Pall.cpu().numpy().reshape(steps + 1, M)[-1]
    assert np.abs(last - out.cpu().numpy()).max() < 1e-9
    del psi
    torch.cuda.empty_cache()
