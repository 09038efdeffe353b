"""The ensemble of Eq. (1) by brute force on the GPU (spin_ensemble_evolve).

Every basis-state member with the polarized site up is evolved on its own
(2^c members at a time, stacked on the top address bits of one state) and
the members' local polarizations are averaged on the device.  Checked
against:
* the oracle's Trotterised ensemble average (``ed.ensemble_P_trotter``,
  sector by sector) over every step at M = 8..12, and on a 3-step prefix of
  the whole 2 x 7 ladder (M = 14);
* member ranges at M = 16, 18 and 20 (2 x 8, 2 x 9, 2 x 10 XY ladders, 100 steps)
  against the mean of the oracle's Trotter loop run on each member's basis
  state, with ragged member counts and evolutions of a few members;
* the whole ensemble of an XY chain at M = 18 (2^17 members): the
  free-fermion closed form |g_00|^2 of the Trotterised single-particle
  propagator at every step;
* the whole ensemble of the 2 x 8, 2 x 9 and 2 x 10 ladders on the first two steps:
  after k Strang steps (list order: even leg bonds, odd leg bonds, rungs)
  site 0's Heisenberg operator reaches leg sites 0..2k+1 only, so the
  ensemble P of any 2 x L ladder with L >= 2k+2 equals that of the 2 x 6
  ladder, which the oracle's ensemble average computes.
Tolerances as every parity test: 1e-10 in FP64, 1e-4 in FP32 on P, and the
same on the mean norm (which is 1).
"""
import functools

import numpy as np
import pytest

import workloads
from oracle import cref, ed
import paper_0710_3747_amd as spq
from gpu_helpers import TOL_P, note, torch_dtype

pytestmark = pytest.mark.gpu
C64, C128 = spq.SPIN_C64, spq.SPIN_C128
PRECS = [C64, C128]


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    spq.load_library()
    cref.build(force=False)
    yield
    torch.cuda.empty_cache()


def gpu_ensemble(prec, M, J, dt, steps, polarized, observed, first=0, count=None,
                 work_members=None, opts=None):
    """(P, N) of spin_ensemble_evolve; the work buffer holds `work_members`
    member states (default: all of them)."""
    import torch
    if count is None:
        count = 2 ** (M - 1) - first
    wm = count if work_members is None else work_members
    work = torch.empty(2 ** M * wm, dtype=torch_dtype(prec), device="cuda")
    P = torch.full((steps + 1,), float("nan"), dtype=torch.float64, device="cuda")
    N = torch.full((steps + 1,), float("nan"), dtype=torch.float64, device="cuda")
    o = spq.Options(**opts) if opts else None
    spq.spin_ensemble_evolve(work, M, J, dt, steps, polarized, observed, P, N, first, count, o)
    torch.cuda.synchronize()
    del work
    torch.cuda.empty_cache()
    return P.cpu().numpy(), N.cpu().numpy()


def member_state(M, polarized, r):
    """Basis index of member r: the bits of r on the sites other than the
    polarized one, in site order; the polarized site's bit is 0 (up)."""
    x, j = 0, 0
    for s in range(M):
        if s == polarized:
            continue
        if (r >> j) & 1:
            x |= 1 << s
        j += 1
    return x


def oracle_member_mean(M, J, dt, steps, polarized, observed, members):
    acc = np.zeros(steps + 1)
    for r in members:
        psi = np.zeros(2 ** M, dtype=np.complex128)
        psi[member_state(M, polarized, r)] = 1.0
        P, _ = cref.trotter_run(psi, M, J, dt, steps, observed)
        acc += P
    return acc / len(members)


@functools.lru_cache(maxsize=None)
def oracle_ensemble(name, M, steps, polarized, observed):
    return ed.ensemble_P_trotter(M, SMALL_J[name], SMALL_DT[name], steps, polarized, observed)


SMALL_J = {
    "ladder_2x4": workloads.ladder(4),
    "ladder_2x5_zz": workloads.ladder(5, a_over_b=0.7),
    "star_12": workloads.star(12, 5),
    "ladder_2x7": workloads.ladder(7),
    "ladder_2x6": workloads.ladder(6),
}
SMALL_DT = {"ladder_2x4": 0.05, "ladder_2x5_zz": 0.07, "star_12": 0.02, "ladder_2x7": 0.05,
            "ladder_2x6": 0.05}
# (workload, M, steps, polarized, observed, members per evolution)
SMALL_CASES = [
    ("ladder_2x4", 8, 60, 0, 0, 8),        # 16 evolutions of 8 members
    ("ladder_2x4", 8, 60, 5, 2, 1),        # one member at a time
    ("ladder_2x5_zz", 10, 50, 3, 6, None),  # one evolution of all 512
    ("star_12", 12, 40, 0, 0, 100),        # 64 per evolution (work for 100), 32 evolutions
    ("ladder_2x7", 14, 3, 0, 0, 1024),     # the whole 2 x 7 ladder, 8 evolutions
]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", PRECS, ids=["c64", "c128"])
@pytest.mark.parametrize("case", SMALL_CASES, ids=lambda c: f"{c[0]}-p{c[3]}o{c[4]}-w{c[5]}")
def test_ensemble_matches_oracle_ensemble(prec, case):
    name, M, steps, pol, obs, wm = case
    note("ensemble", name, prec, case)
    P, N = gpu_ensemble(prec, M, SMALL_J[name], SMALL_DT[name], steps, pol, obs, work_members=wm)
    want = oracle_ensemble(name, M, steps, pol, obs)
    assert np.abs(P - want).max() < TOL_P[prec], np.abs(P - want).max()
    assert np.abs(N - 1).max() < TOL_P[prec]


# (L, polarized, observed, [(first, count)], members per evolution)
RANGE_CASES = [
    (8, 0, 0, [(0, 5), (2 ** 14 - 3, 7), (2 ** 15 - 4, 4)], 2),
    (8, 3, 0, [(1000, 9)], 4),
    (9, 0, 0, [(0, 3), (2 ** 16 + 11, 5), (2 ** 17 - 6, 6)], 4),
    (10, 7, 0, [(0, 2), (2 ** 19 - 5, 5)], 2),
]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", PRECS, ids=["c64", "c128"])
@pytest.mark.parametrize("case", RANGE_CASES, ids=lambda c: f"2x{c[0]}-p{c[1]}o{c[2]}")
def test_member_ranges_match_member_runs(prec, case):
    """Member ranges at M = 16, 18 and 20 against the oracle loop on each
    member's basis state, 100 steps."""
    L, pol, obs, ranges, wm = case
    M, J, dt, steps = 2 * L, workloads.ladder(L), 0.05, 100
    for first, count in ranges:
        note("ensemble range", M, prec, first, count)
        P, N = gpu_ensemble(prec, M, J, dt, steps, pol, obs, first, count, work_members=wm)
        want = oracle_member_mean(M, J, dt, steps, pol, obs, range(first, first + count))
        assert np.abs(P - want).max() < TOL_P[prec], (first, count, np.abs(P - want).max())
        assert np.abs(N - 1).max() < TOL_P[prec]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", PRECS, ids=["c64", "c128"])
def test_whole_ensemble_xy_chain_M18_free_fermions(prec):
    """All 2^17 members of an 18-site XY chain, 40 steps: the ensemble P of
    the end site is |g_00|^2 of the Trotterised single-particle propagator."""
    M, dt, steps = 18, 0.05, 40
    J = workloads.chain(M)
    note("ensemble chain 18", prec)
    P, N = gpu_ensemble(prec, M, J, dt, steps, 0, 0, work_members=2 ** 14)
    bonds = [(i, j, b) for (i, j, a, b) in J]
    want = ed.free_fermion_P(M, bonds, dt=dt, n_steps=steps)
    assert np.abs(P - want).max() < TOL_P[prec], np.abs(P - want).max()
    assert np.abs(N - 1).max() < TOL_P[prec]
    assert want[-1] < 0.7      # the closed form has moved well away from 1


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", PRECS, ids=["c64", "c128"])
@pytest.mark.parametrize("L", [8, 9, 10])
def test_whole_ladder_ensemble_two_steps_light_cone(prec, L):
    """The whole ensemble of the 2 x L ladder (M = 16, 18, 20; 2^19 members
    at M = 20) after 0..2 steps equals the oracle's ensemble of the 2 x 6
    ladder (light cone)."""
    M, steps = 2 * L, 2
    note("ensemble light cone", M, prec)
    P, N = gpu_ensemble(prec, M, workloads.ladder(L), 0.05, steps, 0, 0, work_members=2 ** 12)
    want = oracle_ensemble("ladder_2x6", 12, steps, 0, 0)
    assert np.abs(P - want).max() < TOL_P[prec], np.abs(P - want).max()
    assert np.abs(N - 1).max() < TOL_P[prec]
    assert want[-1] < 1 - 1e-3


def test_ensemble_equals_batched_basis_members():
    """The stacked evolution and the batched launch of SPIN_INIT_BASIS
    members agree on the 2 x 5 ladder (every member, 80 steps, FP64)."""
    import torch
    M, J, dt, steps = 10, workloads.ladder(5), 0.05, 80
    note("ensemble vs batch", M)
    P, _ = gpu_ensemble(C128, M, J, dt, steps, 0, 0, work_members=64)
    xs = [member_state(M, 0, r) for r in range(2 ** (M - 1))]
    big = torch.empty(len(xs), 2 ** M, dtype=torch.complex128, device="cuda")
    Pb = torch.zeros(len(xs), steps + 1, dtype=torch.float64, device="cuda")
    probs = [dict(psi=big[i], M=M, couplings=J, observed_site=0, seed=x, P=Pb[i])
             for i, x in enumerate(xs)]
    spq.spin_trotter_evolve_batch(probs, C128, dt, steps, init=spq.SPIN_INIT_BASIS)
    assert spq.spin_batch_status() == 0
    assert np.abs(P - Pb.cpu().numpy().mean(0)).max() < 1e-12


def test_ensemble_is_deterministic_and_chunking_invariant():
    """Equal calls give equal bits; other evolution sizes change only the
    summation order (FP64, 2 x 8 ladder, 20 steps)."""
    M, J, dt, steps = 16, workloads.ladder(8), 0.05, 20
    note("ensemble chunking", M)
    a, _ = gpu_ensemble(C128, M, J, dt, steps, 0, 0, work_members=2 ** 10)
    b, _ = gpu_ensemble(C128, M, J, dt, steps, 0, 0, work_members=2 ** 10)
    c, _ = gpu_ensemble(C128, M, J, dt, steps, 0, 0, work_members=3 * 2 ** 12)
    assert np.array_equal(a, b)
    assert np.abs(a - c).max() < 1e-12


@pytest.mark.parametrize("prec", PRECS, ids=["c64", "c128"])
def test_ensemble_tiny_closed_forms(prec):
    """M = 1: the one member keeps P = 1.  M = 2 with one XY bond b: member
    |up, up> keeps P = 1 and |up, down> has P = cos(b t), so the ensemble
    P(t) = (1 + cos(b t)) / 2 (section "Spin systems with different coupling
    networks", single pair); the Strang step is exact for one factor."""
    note("ensemble tiny", prec)
    P, N = gpu_ensemble(prec, 1, [], 0.1, 5, 0, 0)
    assert np.abs(P - 1).max() < TOL_P[prec] and np.abs(N - 1).max() < TOL_P[prec]
    b, dt, steps = 1.3, 0.07, 60
    for pol, obs in ((0, 0), (1, 1)):
        P, N = gpu_ensemble(prec, 2, [(0, 1, 0.0, b)], dt, steps, pol, obs, work_members=1)
        t = dt * np.arange(steps + 1)
        assert np.abs(P - 0.5 * (1 + np.cos(b * t))).max() < TOL_P[prec]
    # observing the partner site: member |up, up> gives +1, member
    # |up, down> gives -cos(b t), so P(t) = (1 - cos(b t)) / 2
    P, N = gpu_ensemble(prec, 2, [(0, 1, 0.0, b)], dt, steps, 0, 1, work_members=2)
    assert np.abs(P - 0.5 * (1 - np.cos(b * t))).max() < TOL_P[prec]


ENSEMBLE_OPTS = [{"schedule": 1}, {"exchange": 1, "tile_bits": 13}, {"use_graph": 1},
                 {"tile_bits": 12, "reg_bits": 4}]


@pytest.mark.parametrize("prec", PRECS, ids=["c64", "c128"])
@pytest.mark.parametrize("opts", ENSEMBLE_OPTS, ids=lambda o: "-".join(f"{k}{v}" for k, v in o.items()))
def test_ensemble_options_reach_the_evolutions(prec, opts):
    """Launch options pass through to the stacked evolutions: the unfused
    schedule, whole-tile exchanges, graph replay and small tiles all give the
    oracle's ensemble (2 x 5 ladder with ZZ, polarised site 3, observed 6;
    64 members per evolution, 8 evolutions)."""
    name, M, steps, pol, obs = "ladder_2x5_zz", 10, 30, 3, 6
    note("ensemble options", prec, opts)
    P, N = gpu_ensemble(prec, M, SMALL_J[name], SMALL_DT[name], steps, pol, obs, work_members=64,
                        opts=opts)
    want = oracle_ensemble(name, M, steps, pol, obs)
    assert np.abs(P - want).max() < TOL_P[prec], np.abs(P - want).max()
    assert np.abs(N - 1).max() < TOL_P[prec]
