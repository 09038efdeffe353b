"""Parity of the HIP path with the CPU oracle, element by element.

Small and mid sizes (several tiles, every kernel path, edge cases).  FP64
states must match the oracle's Trotter loop within 1e-10 on every P[k]
and every amplitude; FP32 states within 1e-4 on P[k] (amplitudes within
1e-4 of the largest).
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle import cref, ed
import paper_0710_3747_amd as spq
from gpu_helpers import TOL_P, assert_state_close, gpu_evolve, gpu_state, note, torch_dtype

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
    torch.cuda.synchronize()


def oracle_run(M, J, dt, steps, obs, pol=0, seed=1, psi0=None):
    psi = oracle.random_phase_state(M, pol, seed) if psi0 is None else psi0.astype(np.complex128).copy()
    psi = np.ascontiguousarray(psi)
    P, N = cref.trotter_run(psi, M, J, dt, steps, obs)
    return P, N, psi


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("M,n,seed", [(1, 0, 3), (2, 1, 0), (7, 3, 2 ** 64 - 1), (14, 13, 5), (21, 0, 99)])
def test_init_matches_oracle(prec, M, n, seed):
    note("init", prec, M, n, seed)
    import torch
    psi = gpu_state(prec, M, n, seed)
    torch.cuda.synchronize()
    got = psi.cpu().numpy().astype(np.complex128)
    want = oracle.random_phase_state(M, n, seed)
    tol = 1e-15 if prec == C128 else 1e-7
    assert np.abs(got - want).max() <= tol * np.abs(want).max() * 4


def test_init_phase_golden_vectors():
    """Phases of the GPU state reproduce stored generator outputs."""
    import os
    import torch
    rows = [l.split() for l in open(os.path.join(os.path.dirname(__file__), "golden", "phase_vectors.txt"))
            if not l.startswith("#")]
    M = 13
    for seed in sorted({int(r[0]) for r in rows})[:4]:
        psi = gpu_state(C128, M, 0, seed)
        torch.cuda.synchronize()
        got = psi.cpu().numpy()
        for s, r, _, u in rows:
            if int(s) != seed or int(r) >= 2 ** (M - 1):
                continue
            x = int(r) << 1          # polarised site 0: x = r with a 0 inserted at bit 0
            phi = 2 * np.pi * float(u)
            assert abs(got[x] * np.sqrt(2.0 ** (M - 1)) - np.exp(1j * phi)) < 1e-13


@pytest.mark.parametrize("prec", PRECS)
def test_local_polarization(prec):
    import torch
    M = 17
    psi0 = oracle.random_phase_state(M, 4, 8)
    psi0 = psi0 * np.exp(0.3j * (np.arange(2 ** M) % 7))  # any state
    rng = np.random.default_rng(0)
    psi0 = psi0 + 1e-3 * (rng.standard_normal(2 ** M) + 1j * rng.standard_normal(2 ** M))
    psi = gpu_state(prec, M, psi0=psi0)
    # guard entries after the outputs: the calls write exactly one value each
    out = torch.full((4,), 7.0, dtype=torch.float64, device="cuda")
    for site in (0, 4, 16):
        note("observe", prec, site)
        spq.spin_local_polarization(psi, M, site, out[0:1])
        spq.spin_local_polarization_ex(psi, M, site, out[1:2], out[2:3])
        torch.cuda.synchronize()
        ref_state = psi.cpu().numpy().astype(np.complex128)
        P, P2, N, guard = out.cpu().numpy()
        assert abs(P - oracle.local_polarization(ref_state, M, site)) < 1e-12
        assert P2 == P and guard == 7.0
        assert abs(N - oracle.norm2(ref_state)) < 1e-12
        spq.spin_local_polarization_ex(psi, M, site, out[3:4], None)
        torch.cuda.synchronize()
        assert float(out[3]) == P
        out[3] = 7.0


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("M", [10, 16])
def test_nan_written_from_the_host_shows_in_P_and_N(prec, M):
    """Failure detection: a NaN put into one amplitude of the state on the
    host (then copied to the device) shows up in P[k] and N[k] of every
    step, in spin_local_polarization and in a batched run -- the
    one-workgroup path (M = 10) and the tiled path (M = 16)."""
    import torch
    J = workloads.ladder(M // 2)
    psi0 = oracle.random_phase_state(M, 0, 3)
    psi0[2 * 77] = complex(float("nan"), 0.0)
    note("nan injection", prec, M)
    P, N, _, t = gpu_evolve(prec, M, J, 0.05, 6, 0, psi0=psi0, keep_state=False)
    assert np.isnan(P).all() and np.isnan(N).all()
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    spq.spin_local_polarization_ex(t, M, 0, out[0:1], out[1:2])
    torch.cuda.synchronize()
    assert np.isnan(out.cpu().numpy()).all()
    Pb = torch.zeros(7, dtype=torch.float64, device="cuda")
    psib = torch.from_numpy(psi0).to(torch_dtype(prec)).cuda()
    spq.spin_trotter_evolve_batch([dict(psi=psib, M=M, couplings=J, observed_site=0, P=Pb)], prec,
                                  0.05, 6, init_random_phase=False)
    assert spq.spin_batch_status() == 0
    assert np.isnan(Pb.cpu().numpy()).all()


@pytest.mark.parametrize("prec", PRECS)
def test_config_ladder_2x5_full(prec):
    """Ladder 2x5, J = 1, dt = 0.05, 400 steps, site 0 polarised (whole
    state in one workgroup)."""
    M, (L, dt, steps, seed) = 10, workloads.LADDER_CONFIGS["ladder_2x5"]
    J = workloads.ladder(L)
    note("ladder 2x5", prec)
    P, N, psi, _ = gpu_evolve(prec, M, J, dt, steps, 0, seed=seed)
    Pw, Nw, psiw = oracle_run(M, J, dt, steps, 0, seed=seed)
    assert np.abs(P - Pw).max() < TOL_P[prec]
    assert np.abs(N - Nw).max() < TOL_P[prec]
    assert_state_close(psi, psiw, prec)


TILED = [
    # name, M, couplings, dt, steps, observed, polarized, options
    ("ladder16", 16, workloads.ladder(8), 0.05, 25, 0, 0, {}),
    ("ladder16-k12", 16, workloads.ladder(8), 0.05, 25, 0, 0, {"tile_bits": 12}),
    ("ladder18-periodic", 18, workloads.ladder(9), 0.05, 110, 0, 0, {}),
    ("star16-k13", 16, workloads.star(16, 4), 0.02, 8, 0, 0, {"tile_bits": 13}),
    ("star15-zz-obs3", 15, workloads.star(15, 5, a_over_b=-2.0), 0.03, 6, 3, 1, {}),
    ("mixed17-r4", 17, workloads.ladder(8, a_over_b=0.7) + [(2, 16, 0.3, -1.1), (0, 16, 0.0, 0.4)],
     0.05, 10, 16, 16, {"reg_bits": 4, "tile_bits": 12}),
    ("uncoupled-observed-periodic", 16, [(1, 2, 0.0, 1.0), (5, 15, 0.0, 1.0)], 0.1, 100, 0, 0, {}),
    ("no-couplings", 15, [], 0.1, 5, 3, 0, {}),
    ("large-angles", 15, [(0, 1, 3.0, 40.0), (1, 14, 0.0, -35.0), (3, 9, 0.0, 100.0)], 0.1, 6, 0, 0, {}),
    ("duplicate-pairs", 15, workloads.chain(15) + [(0, 1, 0.0, 1.0), (1, 0, 0.0, 0.5)], 0.05, 12, 1, 0, {}),
    # 128-byte runs (complex64: 16 amplitudes), 512 and 1024 lanes
    ("ladder20-c4", 20, workloads.ladder(10), 0.05, 30, 0, 0, {"coalesce_bits": 4}),
    ("ladder20-r4-c4", 20, workloads.ladder(10), 0.05, 30, 0, 0, {"reg_bits": 4, "coalesce_bits": 4}),
    # tiles of 2^14 amplitudes with half-tile exchanges (complex128: one
    # 512-lane workgroup per CU, 32 amplitudes per lane)
    ("ladder20-k14", 20, workloads.ladder(10), 0.05, 30, 0, 0, {"tile_bits": 14, "coalesce_bits": 4}),
    ("star17-k14-zz", 17, workloads.star(17, 8, a_over_b=-2.0), 0.02, 6, 2, 5, {"tile_bits": 14}),
]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", TILED, ids=[c[0] for c in TILED])
def test_tiled_path_matches_oracle(prec, case):
    name, M, J, dt, steps, obs, pol, opts = case
    if prec == C128 and opts.get("tile_bits", 0) > 14:
        pytest.skip("complex128 tiles hold at most 2^14 amplitudes")
    if prec == C64 and opts.get("reg_bits") == 4 and opts.get("tile_bits") not in (None, 12):
        pytest.skip("no such complex64 shape")
    note("tiled", name, prec)
    info = spq.spin_describe_plan(prec, M, J, dt, steps, obs, spq.Options(**opts))
    assert info["path"] == 2
    P, N, psi, _ = gpu_evolve(prec, M, J, dt, steps, obs, polarized=pol, seed=7, opts=opts)
    Pw, Nw, psiw = oracle_run(M, J, dt, steps, obs, pol=pol, seed=7)
    assert np.abs(P - Pw).max() < TOL_P[prec]
    assert np.abs(N - Nw).max() < TOL_P[prec]
    assert_state_close(psi, psiw, prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("M", [1, 2, 3, 6, 11, 13, 14])
def test_small_states_one_workgroup(prec, M):
    """Every size of the one-workgroup path, including M = 1 (no bonds)."""
    if prec == C128 and M == 14:
        M = 13
    J = [(i, j, 0.0, 1.0) for i in range(M) for j in range(i + 1, M) if (i + j) % 3 != 1][: 3 * M]
    note("small", prec, M, len(J))
    P, N, psi, _ = gpu_evolve(prec, M, J, 0.07, 30, 0, seed=M)
    Pw, Nw, psiw = oracle_run(M, J, 0.07, 30, 0, seed=M)
    assert np.abs(P - Pw).max() < TOL_P[prec]
    assert_state_close(psi, psiw, prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("M,j", [(2, 1), (16, 15), (20, 19)])
def test_single_bond_closed_form(prec, M, j):
    """Only bond (0, j): P(t) = (1 + cos(b t))/2 exactly (any a, seed, dt)."""
    b, dt, steps = 1.7, 0.05, 120
    note("single bond", prec, M, j)
    P, N, _, _ = gpu_evolve(prec, M, [(0, j, 0.4, b)], dt, steps, 0, seed=3, keep_state=False)
    k = np.arange(steps + 1)
    assert np.abs(P - 0.5 * (1 + np.cos(b * k * dt))).max() < TOL_P[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_unfused_schedule_matches_oracle_and_fused(prec):
    M, J = 15, workloads.ladder(7) + [(0, 14, 0.5, 0.8)]
    note("unfused", prec)
    Pu, _, psiu, _ = gpu_evolve(prec, M, J, 0.05, 8, 0, opts={"schedule": 1})
    Pf, _, psif, _ = gpu_evolve(prec, M, J, 0.05, 8, 0)
    Pw, _, psiw = oracle_run(M, J, 0.05, 8, 0)
    assert np.abs(Pu - Pw).max() < TOL_P[prec] and np.abs(Pf - Pw).max() < TOL_P[prec]
    assert_state_close(psiu, psiw, prec)


@pytest.mark.parametrize("prec", PRECS)
def test_zero_steps_and_time_reversal(prec):
    M, J = 16, workloads.star(16, 9)
    note("reversal", prec)
    P0, _, psi_same, _ = gpu_evolve(prec, M, J, 0.05, 0, 0, seed=4)
    psi0 = oracle.random_phase_state(M, 0, 4)
    assert_state_close(psi_same, psi0, prec)
    assert abs(P0[0] - 1) < TOL_P[prec]
    _, _, _, t = gpu_evolve(prec, M, J, 0.05, 20, 0, seed=4, keep_state=False)
    _, _, back, _ = gpu_evolve(prec, M, J, -0.05, 20, 0, psi=t)
    assert np.abs(back - psi0).max() < (1e-12 if prec == C128 else 1e-5) * np.abs(psi0).max() * 100


@pytest.mark.parametrize("prec", PRECS)
def test_determinism_bitwise(prec):
    M, J = 17, workloads.ladder(8) + [(0, 16, 0.0, 1.0)]
    note("determinism", prec)
    P1, N1, s1, _ = gpu_evolve(prec, M, J, 0.05, 30, 0, seed=2)
    P2, N2, s2, _ = gpu_evolve(prec, M, J, 0.05, 30, 0, seed=2)
    assert np.array_equal(P1, P2) and np.array_equal(N1, N2) and np.array_equal(s1, s2)


@pytest.mark.parametrize("prec", PRECS)
def test_chunked_run_equals_single_run(prec):
    """Resuming from the state buffer (two calls) gives the same dynamics."""
    M, J = 16, workloads.ladder(8)
    note("chunked", prec)
    P, _, psi, _ = gpu_evolve(prec, M, J, 0.05, 60, 0, seed=6)
    Pa, _, _, t = gpu_evolve(prec, M, J, 0.05, 25, 0, seed=6, keep_state=False)
    Pb, _, psib, _ = gpu_evolve(prec, M, J, 0.05, 35, 0, psi=t)
    assert np.abs(np.concatenate([Pa, Pb[1:]]) - P).max() < TOL_P[prec]
    assert_state_close(psib, psi, prec)


@pytest.mark.parametrize("prec", PRECS)
def test_batch_matches_single_runs(prec):
    import torch
    probs_spec = workloads.star_batch(12, 5, 13 if prec == C128 else 14, 4, 500, 600)
    steps, dt = 40, 0.02
    probs = []
    for r, p in enumerate(probs_spec):
        M = p["M"]
        probs.append(dict(psi=torch.empty(2 ** M, dtype=torch.complex64 if prec == C64 else torch.complex128,
                                          device="cuda"),
                          M=M, couplings=p["couplings"], observed_site=0, polarized_site=0, seed=p["seed"],
                          P=torch.zeros(steps + 1, dtype=torch.float64, device="cuda"),
                          N=torch.zeros(steps + 1, dtype=torch.float64, device="cuda")))
    note("batch", prec, [p["M"] for p in probs])
    spq.spin_trotter_evolve_batch(probs, prec, dt, steps, init_random_phase=True)
    assert spq.spin_batch_status() == 0, spq.spin_last_error()
    torch.cuda.synchronize()
    for p in probs:
        # problems held in LDS use the batch's register stages and the
        # largest ones run as a one-workgroup gang of tiled passes, so the
        # rotations' shears may run in the other order of a pair: equal to
        # rounding
        P, N, psi, _ = gpu_evolve(prec, p["M"], p["couplings"], dt, steps, 0, seed=p["seed"])
        assert np.abs(p["P"].cpu().numpy() - P).max() < TOL_P[prec]
        assert_state_close(p["psi"].cpu().numpy().astype(np.complex128), psi, prec)
    # and one against the oracle
    p = probs[0]
    Pw, _, psiw = oracle_run(p["M"], p["couplings"], dt, steps, 0, seed=p["seed"])
    assert np.abs(p["P"].cpu().numpy() - Pw).max() < TOL_P[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_batch_gangs_match_single_runs(prec):
    """Problems larger than one workgroup run as gangs of workgroups inside
    the persistent launch.  Where the single-problem path runs the same plan
    (tiled, at the gangs' launch shape) states must agree bit for bit and P
    to FP64 rounding; the others (held in LDS, or one tile run as a gang of
    one) agree to the parity tolerances."""
    import torch
    Ms = [15, 14, 16, 17, 18, 6, 15]
    steps, dt = 30, 0.02
    probs = []
    for r, M in enumerate(Ms):
        probs.append(dict(psi=torch.empty(2 ** M, dtype=torch.complex64 if prec == C64 else torch.complex128,
                                          device="cuda"),
                          M=M, couplings=workloads.star(M, 300 + r), observed_site=0, polarized_site=0,
                          seed=700 + r, P=torch.zeros(steps + 1, dtype=torch.float64, device="cuda"),
                          N=torch.zeros(steps + 1, dtype=torch.float64, device="cuda")))
    note("batch gangs", prec, Ms)
    spq.spin_trotter_evolve_batch(probs, prec, dt, steps, init_random_phase=True)
    assert spq.spin_batch_status() == 0, spq.spin_last_error()
    torch.cuda.synchronize()
    for p in probs:
        # the gangs' launch shape: 64 amplitudes per lane (32 in complex128)
        # with half-tile exchanges
        shape = (14, 6, 4) if prec == C64 else (13, 5, 4)
        P, N, psi, _ = gpu_evolve(prec, p["M"], p["couplings"], dt, steps, 0, seed=p["seed"],
                                  opts=dict(zip(("tile_bits", "reg_bits", "coalesce_bits"), shape)))
        got = p["psi"].cpu().numpy().astype(np.complex128)
        if p["M"] > shape[0]:
            assert np.abs(p["P"].cpu().numpy() - P).max() < 1e-13
            assert np.array_equal(got, psi)
        else:
            assert np.abs(p["P"].cpu().numpy() - P).max() < TOL_P[prec]
            assert_state_close(got, psi, prec)
    p = probs[0]
    Pw, _, psiw = oracle_run(p["M"], p["couplings"], dt, steps, 0, seed=p["seed"])
    assert np.abs(p["P"].cpu().numpy() - Pw).max() < TOL_P[prec]
    # a second call with the same problems reuses the cached launch
    spq.spin_trotter_evolve_batch(probs, prec, dt, steps, init_random_phase=True)
    assert spq.spin_batch_status() == 0, spq.spin_last_error()
    torch.cuda.synchronize()
    assert np.abs(probs[0]["P"].cpu().numpy() - Pw).max() < TOL_P[prec]


def test_batch_config_256_uneven_stars():
    """256 stars, M uniform in 14..20, couplings as the M = 28 star, 500
    steps at dt = 0.02, complex64, one persistent launch."""
    import torch
    cfg = workloads.BATCH_STARS
    spec = workloads.star_batch(cfg["n"], cfg["m_lo"], cfg["m_hi"], cfg["size_seed"],
                                cfg["coupling_seed0"], cfg["state_seed0"])
    steps, dt = cfg["n_steps"], cfg["dt"]
    probs = []
    for p in spec:
        probs.append(dict(psi=torch.empty(2 ** p["M"], dtype=torch.complex64, device="cuda"),
                          M=p["M"], couplings=p["couplings"], observed_site=0, polarized_site=0,
                          seed=p["seed"], P=torch.zeros(steps + 1, dtype=torch.float64, device="cuda"),
                          N=torch.zeros(steps + 1, dtype=torch.float64, device="cuda")))
    note("batch 256 stars")
    spq.spin_trotter_evolve_batch(probs, C64, dt, steps, init_random_phase=True)
    assert spq.spin_batch_status() == 0, spq.spin_last_error()
    torch.cuda.synchronize()
    for p in probs:
        P, N = p["P"].cpu().numpy(), p["N"].cpu().numpy()
        assert np.isfinite(P).all() and abs(P[0] - 1) < 1e-6
        assert np.abs(N - 1).max() < 1e-4
    # the single path searches scheduling variants for calls this long, the
    # batch takes the default one: the same product, grouped differently,
    # so the two agree to FP32 rounding
    picks = [int(np.argmin([p["M"] for p in probs])), 7, int(np.argmax([p["M"] for p in probs]))]
    for i in picks:
        p = probs[i]
        P, _, _, _ = gpu_evolve(C64, p["M"], p["couplings"], dt, steps, 0, seed=p["seed"], keep_state=False)
        assert np.abs(p["P"].cpu().numpy() - P).max() < 2e-5
    p = probs[picks[0]]     # the oracle on a smallest problem, full run
    Pw, _, _ = oracle_run(p["M"], p["couplings"], dt, steps, 0, seed=p["seed"])
    assert np.abs(p["P"].cpu().numpy() - Pw).max() < TOL_P[C64]


_BATCH_ORACLE = {}


def _batch_subset(spec):
    """A seeded subset of the 256-star batch: one problem of each size
    15..19 and two of size 20 (the gangs of 2..32 workgroups)."""
    rng = np.random.default_rng(20)
    out = []
    for M, n in ((15, 1), (16, 1), (17, 1), (18, 1), (19, 1), (20, 2)):
        idx = [i for i, p in enumerate(spec) if p["M"] == M]
        out += [int(i) for i in rng.choice(idx, size=n, replace=False)]
    return out


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", [C64, C128], ids=["c64", "c128"])
def test_batch_config_256_gang_problems_match_oracle(prec):
    """256 stars (M uniform in 14..20), 500 steps at dt = 0.02, one
    persistent launch in each precision: a seeded subset of the problems run
    by gangs (one of each size 15..19, two of size 20) against the oracle's
    loop over all 500 steps -- every P[k], N[k] and the final state; the
    phase-draw mean of Eq. (4) averages such problems."""
    import torch
    cfg = workloads.BATCH_STARS
    spec = workloads.star_batch(cfg["n"], cfg["m_lo"], cfg["m_hi"], cfg["size_seed"],
                                cfg["coupling_seed0"], cfg["state_seed0"])
    steps, dt = cfg["n_steps"], cfg["dt"]
    probs = []
    for p in spec:
        probs.append(dict(psi=torch.empty(2 ** p["M"], dtype=torch_dtype(prec), device="cuda"),
                          M=p["M"], couplings=p["couplings"], observed_site=0, polarized_site=0,
                          seed=p["seed"], P=torch.zeros(steps + 1, dtype=torch.float64, device="cuda"),
                          N=torch.zeros(steps + 1, dtype=torch.float64, device="cuda")))
    note("batch 256 stars vs oracle", prec)
    spq.spin_trotter_evolve_batch(probs, prec, dt, steps, init_random_phase=True)
    assert spq.spin_batch_status() == 0, spq.spin_last_error()
    for i in _batch_subset(spec):
        p = probs[i]
        if i not in _BATCH_ORACLE:
            note("oracle star", i, "M", p["M"])
            _BATCH_ORACLE[i] = oracle_run(p["M"], p["couplings"], dt, steps, 0, seed=p["seed"])
        Pw, Nw, psiw = _BATCH_ORACLE[i]
        P, N = p["P"].cpu().numpy(), p["N"].cpu().numpy()
        assert np.abs(P - Pw).max() < TOL_P[prec], (i, p["M"], np.abs(P - Pw).max())
        assert np.abs(N - Nw).max() < TOL_P[prec], (i, p["M"])
        assert_state_close(p["psi"].cpu().numpy().astype(np.complex128), psiw, prec)


def test_autotune_picks_a_shape_stores_it_and_it_evolves_correctly(tmp_path):
    """The autotuner times every candidate shape, keeps the fastest in the
    process cache and the JSON file, and the tuned options give the oracle's
    result."""
    import json
    M, J, dt, steps = 18, workloads.ladder(9), 0.05, 12
    path = str(tmp_path / "tune.json")
    note("autotune M=18")
    out = spq.spin_autotune(C64, M, J, dt, 0, trial_steps=6, cache_path=path)
    res = out["results"]
    assert len(res) >= 4 and all(r["status"] == 0 and r["ms_per_step"] > 0 for r in res)
    best = out["best"]
    fastest = min(res, key=lambda r: r["ms_per_step"])
    assert (best.tile_bits, best.reg_bits, best.coalesce_bits) == \
        (fastest["tile_bits"], fastest["reg_bits"], fastest["coalesce_bits"])
    entries = json.load(open(path))["entries"]
    assert len(entries) == 1 and list(entries.values())[0]["tile_bits"] == best.tile_bits
    got = spq.spin_tuned_options(C64, M, J, dt, 0)
    assert got is not None and got.tile_bits == best.tile_bits
    spq.spin_release_caches()
    assert spq.spin_tuned_options(C64, M, J, dt, 0) is None
    got = spq.spin_tuned_options(C64, M, J, dt, 0, cache_path=path)
    assert got is not None and (got.tile_bits, got.reg_bits) == (best.tile_bits, best.reg_bits)
    assert spq.spin_tuned_options(C64, M, J, 2 * dt, 0, cache_path=path) is None
    P, N, psi, _ = gpu_evolve(C64, M, J, dt, steps, 0, seed=3,
                              opts={"tile_bits": got.tile_bits, "reg_bits": got.reg_bits,
                                    "coalesce_bits": got.coalesce_bits})
    psi0 = oracle.random_phase_state(M, 0, 3)
    Pw, Nw, psiw = oracle.trotter_run(psi0, M, J, dt, steps, 0)
    assert np.abs(P - Pw).max() < TOL_P[C64]
    assert_state_close(psi, psiw, C64)


@pytest.mark.parametrize("M,steps,a_over_b", [(18, 12, 0.0), (20, 9, -2.0), (16, 40, 0.5)])
def test_mfma_engine_matches_oracle(M, steps, a_over_b):
    """Matrix engine: each stage's factors fused into one 32 x 32 complex
    matrix applied on FP32 MFMA; state and P against the oracle (FP32
    tolerance), with and without I^z I^z terms, over several tiles."""
    J = workloads.ladder(M // 2, a_over_b=a_over_b)
    opts = {"engine": 1}
    info = spq.spin_describe_plan(C64, M, J, 0.05, steps, 0, spq.Options(**opts))
    assert info["path"] == 2 and info["engine"] == 1
    note("mfma engine", M, steps, a_over_b)
    P, N, psi, _ = gpu_evolve(C64, M, J, 0.05, steps, 0, seed=4, opts=opts)
    psi0 = oracle.random_phase_state(M, 0, 4)
    Pw, Nw, psiw = oracle.trotter_run(psi0, M, J, 0.05, steps, 0)
    assert np.abs(P - Pw).max() < TOL_P[C64]
    assert np.abs(N - 1).max() < 1e-4
    assert_state_close(psi, psiw, C64)


@pytest.mark.parametrize("prec", PRECS)
def test_ensemble_of_basis_states_matches_trotterised_ensemble(prec):
    """The literal ensemble of Eq. (1) on the GPU: all 2^9 basis states of the
    2 x 5 ladder with site 0 up, each evolved 400 steps in one batched launch
    (SPIN_INIT_BASIS), averaged; against the oracle's Trotterised ensemble
    (sector step matrices, FP64)."""
    import torch
    M, (L, dt, steps, seed) = 10, workloads.LADDER_CONFIGS["ladder_2x5"]
    J = workloads.ladder(L)
    xs = [x for x in range(2 ** M) if not (x & 1)]
    dtype = torch.complex64 if prec == C64 else torch.complex128
    note("basis ensemble 2x5", prec)
    probs = [dict(psi=torch.empty(2 ** M, dtype=dtype, device="cuda"), M=M, couplings=J,
                  observed_site=0, seed=x, P=torch.zeros(steps + 1, dtype=torch.float64, device="cuda"))
             for x in xs]
    spq.spin_trotter_evolve_batch(probs, prec, dt, steps, init=spq.SPIN_INIT_BASIS)
    assert spq.spin_batch_status() == 0, spq.spin_last_error()
    torch.cuda.synchronize()
    Pbar = torch.stack([p["P"] for p in probs]).mean(0).cpu().numpy()
    want = ed.ensemble_P_trotter(M, J, dt, steps, 0, 0)
    assert np.abs(Pbar - want).max() < (1e-10 if prec == C128 else 1e-4)
    # one member against the oracle loop, element by element
    x = xs[37]
    psi0 = np.zeros(2 ** M, dtype=np.complex128)
    psi0[x] = 1.0
    Pw, _, psiw = oracle.trotter_run(psi0, M, J, dt, steps, 0)
    assert np.abs(probs[37]["P"].cpu().numpy() - Pw).max() < TOL_P[prec]
    assert_state_close(probs[37]["psi"].cpu().numpy().astype(np.complex128), psiw, prec)


def test_basis_init_on_the_gang_path():
    """SPIN_INIT_BASIS for states larger than one workgroup (M = 16, gangs of
    workgroups over shared pass tables)."""
    import torch
    M, J, dt, steps = 16, workloads.ladder(8), 0.05, 10
    xs = [0b0000000000000010, 0b0101001000011100, 2 ** 16 - 2]
    note("basis init gangs")
    probs = [dict(psi=torch.empty(2 ** M, dtype=torch.complex128, device="cuda"), M=M, couplings=J,
                  observed_site=3, seed=x, P=torch.zeros(steps + 1, dtype=torch.float64, device="cuda"))
             for x in xs]
    spq.spin_trotter_evolve_batch(probs, C128, dt, steps, init=spq.SPIN_INIT_BASIS)
    assert spq.spin_batch_status() == 0, spq.spin_last_error()
    torch.cuda.synchronize()
    for pr, x in zip(probs, xs):
        psi0 = np.zeros(2 ** M, dtype=np.complex128)
        psi0[x] = 1.0
        Pw, _, psiw = oracle.trotter_run(psi0, M, J, dt, steps, 3)
        assert np.abs(pr["P"].cpu().numpy() - Pw).max() < TOL_P[C128]
        assert_state_close(pr["psi"].cpu().numpy(), psiw, C128)


# ------------------------------------------------------------ all-site profile
PROFILE = [
    # name, M, couplings, dt, steps, polarised site, options
    ("resident-ladder10", 10, workloads.ladder(5), 0.05, 30, 0, {}),
    ("resident-star9-zz", 9, workloads.star(9, 3, a_over_b=-2.0), 0.07, 12, 4, {}),
    ("tiled-ladder16-k12", 16, workloads.ladder(8), 0.05, 12, 0, {"tile_bits": 12}),
    ("tiled-ladder18-long", 18, workloads.ladder(9), 0.05, 60, 0, {}),
    ("tiled-star15-r4", 15, workloads.star(15, 8, a_over_b=1.0), 0.02, 5, 7,
     {"tile_bits": 12, "reg_bits": 4}),
    ("tiled-chain17", 17, workloads.chain(17), 0.1, 20, 0, {}),
    ("unfused-ladder8", 8, workloads.ladder(4), 0.1, 4, 0, {"schedule": 1}),
    ("tiled-ladder16-nomerge-backwards", 16, workloads.ladder(8, a_over_b=0.5), -0.05, 9, 3,
     {"tile_bits": 12, "no_merge": 1}),
    # tiles of 2^14 (complex128: one 512-lane workgroup per CU) and 64
    # amplitudes per lane
    ("tiled-ladder18-k14", 18, workloads.ladder(9), 0.05, 15, 0, {"tile_bits": 14}),
    ("tiled-star16-k14-r6", 16, workloads.star(16, 12), 0.02, 6, 2, {"tile_bits": 14, "reg_bits": 6}),
]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", PROFILE, ids=[c[0] for c in PROFILE])
def test_profile_matches_oracle(prec, case):
    """Every site's polarisation after every step, element by element against
    the oracle's profile loop, plus the norm and the final state."""
    from gpu_helpers import gpu_profile
    name, M, J, dt, steps, pol, opts = case
    if prec == C128 and opts.get("reg_bits") == 6:
        pytest.skip("no complex128 shape with 64 amplitudes per lane")
    note("profile", name, prec)
    Pg, Ng, psig = gpu_profile(prec, M, J, dt, steps, pol, 7, opts)
    Pw, Nw, psiw = oracle.trotter_profile(oracle.random_phase_state(M, pol, 7), M, J, dt, steps)
    assert np.abs(Pg - Pw).max() < TOL_P[prec]
    assert np.abs(Ng - Nw).max() < TOL_P[prec]
    assert_state_close(psig, psiw, prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("M", [1, 2, 3, 5])
def test_profile_smallest_states(prec, M):
    """The whole-state kernel's profile at the smallest sizes (fewer sites
    than register bits), element by element against the oracle."""
    from gpu_helpers import gpu_profile
    J = [] if M == 1 else [(i, (i + 1) % M, 0.4, 1.1) for i in range(M - 1)]
    note("profile small", prec, M)
    Pg, Ng, psig = gpu_profile(prec, M, J, 0.2, 7, M - 1, 3)
    Pw, Nw, psiw = oracle.trotter_profile(oracle.random_phase_state(M, M - 1, 3), M, J, 0.2, 7)
    assert np.abs(Pg - Pw).max() < TOL_P[prec]
    assert np.abs(Ng - Nw).max() < TOL_P[prec]
    assert_state_close(psig, psiw, prec)


@pytest.mark.parametrize("prec", PRECS)
def test_profile_chunked_equals_one_call(prec):
    """Two profile calls of 25 steps continue one state like one call of 50
    (different plans, so equal up to rounding)."""
    import torch
    from gpu_helpers import gpu_profile
    M, J, dt = 18, workloads.ladder(9), 0.05
    note("profile chunked", prec)
    P1, N1, psi1 = gpu_profile(prec, M, J, dt, 50, 0, 4)
    psi = gpu_state(prec, M, 0, 4)
    parts = []
    for _ in range(2):
        Pall = torch.zeros(26 * M, dtype=torch.float64, device="cuda")
        spq.spin_trotter_evolve_profile(psi, M, J, dt, 25, Pall)
        parts.append(Pall)
    torch.cuda.synchronize()
    a, b = (t.cpu().numpy().reshape(26, M) for t in parts)
    P2 = np.concatenate([a, b[1:]])
    # the same state read twice: the first call reads a site once its last
    # factor has run (other sites' factors may follow, exact in exact
    # arithmetic), the second at entry; equal up to the state's rounding
    assert np.abs(a[-1] - b[0]).max() < TOL_P[prec]
    assert np.abs(P2 - P1).max() < TOL_P[prec]
    assert_state_close(psi.cpu().numpy().astype(np.complex128), psi1, prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("M,steps", [(23, 50), (28, 4)])
def test_profile_sparse_couplings_many_steps_per_pass(prec, M, steps):
    """One bond between the end sites: a pass spans many steps, so the norm
    slots per pass (one per step) bound the pass, not the observables.  The
    bond's sites follow (1 +- cos bt)/2, the rest stay at zero."""
    from gpu_helpers import gpu_profile
    b, dt = 0.9, 0.1
    note("profile sparse", prec, M, steps)
    Pall, N, _ = gpu_profile(prec, M, [(0, M - 1, 0.2, b)], dt, steps, 0, 2, keep_state=False)
    c = np.cos(b * np.arange(steps + 1) * dt)
    assert np.abs(Pall[:, 0] - 0.5 * (1 + c)).max() < TOL_P[prec]
    assert np.abs(Pall[:, M - 1] - 0.5 * (1 - c)).max() < TOL_P[prec]
    assert np.abs(Pall[:, 1:M - 1]).max() < TOL_P[prec]
    assert np.abs(N - 1).max() < TOL_P[prec]


def test_profile_rejects_matrix_engine_and_null_output():
    import torch
    psi = gpu_state(C64, 16)
    P = torch.zeros(17 * 3, dtype=torch.float64, device="cuda")
    with pytest.raises(spq.SpinError) as e:
        spq.spin_trotter_evolve_profile(psi, 16, workloads.ladder(8), 0.1, 2, P, None,
                                        spq.Options(engine=1))
    assert e.value.code == spq.SPIN_EUNSUPPORTED
    lib = spq.load_library()
    arr, K = spq._couplings(workloads.ladder(8))
    rc = lib.spin_trotter_evolve_profile(psi.data_ptr(), C64, 16, arr, K, 0.1, 2, None, None,
                                         None, None)
    assert rc == spq.SPIN_EINVAL and "Pall" in spq.spin_last_error()


# ------------------------------------------------------------ product state
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("M,n,seed", [(1, 0, 3), (5, 2, 0), (14, 0, 77), (21, 20, 2 ** 64 - 5)])
def test_init_product_matches_oracle(prec, M, n, seed):
    """The product state of the section "Testing the quantum parallelism"
    (site n up, M-1 single-spin phases), element by element."""
    import torch
    note("init product", prec, M, n, seed)
    psi = torch.empty(2 ** M, dtype=torch_dtype(prec), device="cuda")
    spq.spin_init_product(psi, M, n, seed)
    torch.cuda.synchronize()
    got = psi.cpu().numpy().astype(np.complex128)
    want = oracle.product_state(M, n, oracle.product_phases(M, seed))
    # The GPU sums up to M-1 phases before one sincos; the oracle multiplies
    # M-1 complex factors: both round at ~M ulps of the phase sum (< M).
    tol = 4e-15 * M if prec == C128 else 2e-7
    assert np.abs(got - want).max() <= tol * np.abs(want).max()


@pytest.mark.parametrize("prec", PRECS)
def test_batch_product_init_matches_single_runs(prec):
    """SPIN_INIT_PRODUCT inside the batched launch (states held in LDS and a
    gang) equals spin_init_product followed by spin_trotter_evolve."""
    import torch
    note("batch product init", prec)
    steps, dt = 20, 0.03
    probs, singles = [], []
    for idx, (M, seed) in enumerate([(3, 6), (10, 4), (12, 9), (16, 2), (18, 31)]):
        J = workloads.star(M, 40 + idx)
        pol = idx % M
        psi = torch.zeros(2 ** M, dtype=torch_dtype(prec), device="cuda")
        P = torch.zeros(steps + 1, dtype=torch.float64, device="cuda")
        probs.append(dict(psi=psi, M=M, couplings=J, observed_site=0, P=P, polarized_site=pol,
                          seed=seed))
        ref = torch.empty_like(psi)
        spq.spin_init_product(ref, M, pol, seed)
        Pr = torch.zeros(steps + 1, dtype=torch.float64, device="cuda")
        spq.spin_trotter_evolve(ref, M, J, dt, steps, 0, Pr)
        singles.append((ref, Pr))
    spq.spin_trotter_evolve_batch(probs, prec, dt, steps, init=spq.SPIN_INIT_PRODUCT)
    assert spq.spin_batch_status() == 0, spq.spin_last_error()
    torch.cuda.synchronize()
    for pr, (ref, Pr) in zip(probs, singles):
        assert np.abs(pr["P"].cpu().numpy() - Pr.cpu().numpy()).max() < 2e-5
        assert_state_close(pr["psi"].cpu().numpy().astype(np.complex128),
                           ref.cpu().numpy().astype(np.complex128), prec)


def test_fig3a_entangled_vs_product_states_M14():
    """Fig. 3(a), qualitatively, on the 14-spin ladder with b_y/b_x = 1/10:
    one random entangled state follows the exact ensemble (stored, from the
    oracle's exact diagonalisation) within the O(2^-(M-1)/2) deviation; one
    product state (M-1 phases) does not; the mean of N_alpha = 630 product
    states, run as one batched launch, does (630 (M-1) ~ 2^(M-1))."""
    import os
    import torch
    M, dt, steps = 14, 0.05, 300
    J = workloads.ladder(7, bx=1.0, by=0.1)
    gold = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "ensemble_ladder2x7_by0p1.txt"))
    assert np.allclose(gold[:, 0], dt * np.arange(steps + 1))
    Pens = gold[:, 1]
    sigma = 2.0 ** (-(M - 1) / 2)
    rms = lambda P: float(np.sqrt(np.mean((P - Pens) ** 2)))
    note("fig3a singles")
    ent, prod = [], []
    for seed in range(4):
        Pe, _, _, _ = gpu_evolve(C128, M, J, dt, steps, 0, seed=seed, keep_state=False)
        psi = torch.empty(2 ** M, dtype=torch.complex128, device="cuda")
        spq.spin_init_product(psi, M, 0, seed)
        Pp, _, _, _ = gpu_evolve(C128, M, J, dt, steps, 0, psi=psi, keep_state=False)
        ent.append(rms(Pe))
        prod.append(rms(Pp))
    note("fig3a rms ent", ent, "prod", prod, "sigma", sigma)
    assert max(ent) < 2 * sigma
    assert all(p > 2 * e for p, e in zip(prod, ent))
    assert np.median(prod) > 3 * sigma
    note("fig3a batch of 630 product states")
    probs = []
    for a in range(630):
        probs.append(dict(psi=torch.zeros(2 ** M, dtype=torch.complex64, device="cuda"), M=M,
                          couplings=J, observed_site=0, polarized_site=0, seed=1000 + a,
                          P=torch.zeros(steps + 1, dtype=torch.float64, device="cuda")))
    spq.spin_trotter_evolve_batch(probs, C64, dt, steps, init=spq.SPIN_INIT_PRODUCT)
    assert spq.spin_batch_status() == 0, spq.spin_last_error()
    torch.cuda.synchronize()
    mean = np.mean([p["P"].cpu().numpy() for p in probs], axis=0)
    note("fig3a rms mean630", rms(mean))
    assert rms(mean) < 2 * sigma
    assert rms(mean) < np.median(prod) / 3


@pytest.mark.parametrize("prec", PRECS)
def test_graph_replays_equal_eager_runs(prec):
    """use_graph: the captured launch sequence, replayed several times with
    eager work and synchronisations in between, gives bitwise the eager
    result every time (single-site and all-site profile)."""
    import torch
    M, J, dt, steps = 18, workloads.ladder(9), 0.05, 30
    note("graph replays", prec)
    eager_P, _, eager_psi, _ = gpu_evolve(prec, M, J, dt, steps, 0, seed=6)
    from gpu_helpers import gpu_profile
    eager_Pall, _, eager_psi2 = gpu_profile(prec, M, J, dt, steps, 0, 6)
    psi = torch.empty(2 ** M, dtype=torch_dtype(prec), device="cuda")
    P = torch.zeros(steps + 1, dtype=torch.float64, device="cuda")
    Pall = torch.zeros((steps + 1) * M, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = spq.Options(use_graph=1)
    for rep in range(3):
        spq.spin_init_random_phase(psi, M, 0, 6)
        spq.spin_trotter_evolve_ex(psi, M, J, dt, steps, 0, P, None, g)
        spq.spin_local_polarization(psi, M, 3, out)       # eager work on the same stream
        torch.cuda.synchronize()
        assert np.array_equal(P.cpu().numpy(), eager_P), rep
        assert np.array_equal(psi.cpu().numpy().astype(np.complex128), eager_psi), rep
        spq.spin_init_random_phase(psi, M, 0, 6)
        spq.spin_trotter_evolve_profile(psi, M, J, dt, steps, Pall, None, g)
        torch.cuda.synchronize()
        assert np.array_equal(Pall.cpu().numpy().reshape(steps + 1, M), eager_Pall), rep
        assert np.array_equal(psi.cpu().numpy().astype(np.complex128), eager_psi2), rep


def _random_graph(rng, M):
    J = []
    for _ in range(int(rng.integers(1, 3 * M))):
        i, j = (int(x) for x in rng.integers(0, M, size=2))
        if i != j:
            a = float(rng.uniform(-1, 1)) if rng.integers(3) == 0 else 0.0
            J.append((i, j, a, float(rng.uniform(-2, 2))))
    return J


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("seed", range(4))
def test_random_graphs_match_oracle(prec, seed):
    """Seeded random coupling graphs (any pairs, Ising parts, repeated
    pairs), tiled sizes: P, N and the state against the oracle's loop, and
    the all-site profile against the oracle's profile."""
    from gpu_helpers import gpu_profile
    rng = np.random.default_rng(100 + seed)
    M = int(rng.integers(15, 18))
    J = _random_graph(rng, M)
    obs, pol = int(rng.integers(M)), int(rng.integers(M))
    dt, steps = float(rng.uniform(-0.1, 0.1)), int(rng.integers(3, 10))
    note("random graph", prec, seed, M, len(J), steps)
    P, N, psi, _ = gpu_evolve(prec, M, J, dt, steps, obs, polarized=pol, seed=seed)
    Pw, Nw, psiw = oracle_run(M, J, dt, steps, obs, pol, seed)
    assert np.abs(P - Pw).max() < TOL_P[prec]
    assert_state_close(psi, psiw, prec)
    Pg, _, _ = gpu_profile(prec, M, J, dt, steps, pol, seed, keep_state=False)
    Pp, _, _ = oracle.trotter_profile(oracle.random_phase_state(M, pol, seed), M, J, dt, steps)
    assert np.abs(Pg - Pp).max() < TOL_P[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_batch_random_graphs_match_oracle(prec):
    """A batch of seeded random graphs of uneven size (LDS-held and gang
    problems, random observed and polarised sites) against the oracle's loop,
    problem by problem."""
    import torch
    rng = np.random.default_rng(7)
    steps, dt = 12, 0.04
    probs = []
    for r in range(10):
        M = int(rng.integers(3, 18))
        probs.append(dict(psi=torch.empty(2 ** M, dtype=torch_dtype(prec), device="cuda"), M=M,
                          couplings=_random_graph(rng, M), observed_site=int(rng.integers(M)),
                          polarized_site=int(rng.integers(M)), seed=50 + r,
                          P=torch.zeros(steps + 1, dtype=torch.float64, device="cuda")))
    note("batch random graphs", prec, [p["M"] for p in probs])
    spq.spin_trotter_evolve_batch(probs, prec, dt, steps, init=spq.SPIN_INIT_RANDOM_PHASE)
    assert spq.spin_batch_status() == 0, spq.spin_last_error()
    torch.cuda.synchronize()
    for p in probs:
        Pw, _, psiw = oracle_run(p["M"], p["couplings"], dt, steps, p["observed_site"],
                                 p["polarized_site"], p["seed"])
        assert np.abs(p["P"].cpu().numpy() - Pw).max() < TOL_P[prec], p["M"]
        assert_state_close(p["psi"].cpu().numpy().astype(np.complex128), psiw, prec)


def test_fig3b_dipolar_star_entangled_and_product_states_M14():
    """Fig. 3(b), qualitatively: in the dipolar star (every pair coupled,
    b ~ N(0, 1), a = -2b) the cross terms of Eq. (3) decay, so one
    entangled state follows the stored exact ensemble within
    2 * 2^-(M-1)/2 RMS and even one product state stays within 6 times
    that, unlike the ladder of Fig. 3(a) (test above) where it is off by
    more than 15 times."""
    import os
    import torch
    M, dt, steps = 14, 0.02, 250
    J = workloads.star(M, 77, var_center=1.0, var_other=1.0, a_over_b=-2.0)
    gold = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "ensemble_star14_dipolar.txt"))
    assert np.allclose(gold[:, 0], dt * np.arange(steps + 1))
    Pens = gold[:, 1]
    sigma = 2.0 ** (-(M - 1) / 2)
    rms = lambda P: float(np.sqrt(np.mean((P - Pens) ** 2)))
    ent, prod = [], []
    for seed in range(4):
        Pe, _, _, _ = gpu_evolve(C128, M, J, dt, steps, 0, seed=seed, keep_state=False)
        psi = torch.empty(2 ** M, dtype=torch.complex128, device="cuda")
        spq.spin_init_product(psi, M, 0, seed)
        Pp, _, _, _ = gpu_evolve(C128, M, J, dt, steps, 0, psi=psi, keep_state=False)
        ent.append(rms(Pe))
        prod.append(rms(Pp))
    note("fig3b rms ent", ent, "prod", prod, "sigma", sigma)
    assert max(ent) < 2 * sigma
    assert max(prod) < 6 * sigma
