"""Host-side tests of the C-ABI library (no GPU needed).

* the library loads and exports every entry point include/spin.h declares;
* argument validation returns SPIN_EINVAL with a message;
* the planned schedule realises the Strang product: the executed op order
  reported by spin_plan_trace, replayed with the oracle's exact two-spin
  propagators, reproduces the oracle's plain Trotter loop (P at every step
  and the final state) -- for the one-workgroup path, the tiled path (short
  runs and long runs that use the repeating plan) and the unfused schedule.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import workloads
import paper_0710_3747_amd as spq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "spin.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spin_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = spq.load_library()
    names = declared_functions()
    assert "spin_trotter_evolve" in names and len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert "gfx950" in spq.spin_version()


@pytest.mark.parametrize("kw,frag", [
    (dict(M=0), "M"), (dict(M=40), "M"), (dict(observed=7), "observed"),
    (dict(J=[(0, 0, 0.0, 1.0)]), "i == j"), (dict(J=[(0, 9, 0.0, 1.0)]), "out of range"),
    (dict(J=[(0, 1, float("nan"), 1.0)]), "non-finite"), (dict(dt=float("inf")), "dt"),
    (dict(n_steps=-1), "n_steps"),
])
def test_validation_errors(kw, frag):
    args = dict(M=6, J=[(0, 1, 0.0, 1.0)], dt=0.1, n_steps=3, observed=0)
    args.update(kw)
    with pytest.raises(spq.SpinError) as e:
        spq.spin_describe_plan(spq.SPIN_C64, args["M"], args["J"], args["dt"], args["n_steps"],
                               args["observed"])
    assert e.value.code == spq.SPIN_EINVAL and frag in str(e.value)


def test_evolve_rejects_null_state_before_any_device_work():
    lib = spq.load_library()
    arr = (spq._Coupling * 1)()
    P = ctypes.c_void_p(16)
    rc = lib.spin_trotter_evolve(None, spq.SPIN_C64, 4, arr, 0, 0.1, 1, 0, P, None, None)
    assert rc == spq.SPIN_EINVAL and "psi" in spq.spin_last_error()
    rc = lib.spin_trotter_evolve(ctypes.c_void_p(16), 7, 4, arr, 0, 0.1, 1, 0, P, None, None)
    assert rc == spq.SPIN_EINVAL and "prec" in spq.spin_last_error()
    rc = lib.spin_trotter_evolve(ctypes.c_void_p(24), spq.SPIN_C64, 4, arr, 0, 0.1, 1, 0, P, None, None)
    assert rc == spq.SPIN_EINVAL and "aligned" in spq.spin_last_error()
    rc = lib.spin_init_random_phase(ctypes.c_void_p(16), spq.SPIN_C128, 34, 0, 1, None)
    assert rc == spq.SPIN_EINVAL
    rc = lib.spin_local_polarization(ctypes.c_void_p(16), spq.SPIN_C64, 4, 4, P, None)
    assert rc == spq.SPIN_EINVAL


def replay(trace, psi0, M, observed):
    psi = psi0.copy()
    P = {}
    for kind, a, b, A, B in trace:
        if kind == 1:
            P[int(a)] = oracle.local_polarization(psi, M, observed)
        else:
            oracle.apply_factor(psi, M, int(a), int(b), A, B, 1.0)
    return P, psi


CASES = [
    # name, prec, M, couplings, dt, steps, observed, options
    ("ladder10-resident", spq.SPIN_C128, 10, workloads.ladder(5), 0.05, 40, 0, {}),
    ("star9-zz-resident", spq.SPIN_C64, 9, workloads.star(9, 3, a_over_b=-2.0), 0.07, 15, 2, {}),
    ("ladder16-k12", spq.SPIN_C128, 16, workloads.ladder(8), 0.05, 12, 0, {"tile_bits": 12}),
    ("ladder16-k12-long", spq.SPIN_C128, 16, workloads.ladder(8), 0.05, 130, 0, {"tile_bits": 12}),
    ("ladder18-k14-long", spq.SPIN_C64, 18, workloads.ladder(9), 0.05, 110, 0, {}),
    ("star15-k13", spq.SPIN_C128, 15, workloads.star(15, 7), 0.02, 6, 0, {}),
    ("star15-k12-obs5", spq.SPIN_C64, 15, workloads.star(15, 8, a_over_b=1.0), 0.02, 5, 5,
     {"tile_bits": 12, "reg_bits": 4}),
    ("mixed16-nomerge", spq.SPIN_C64, 16, workloads.ladder(8, a_over_b=0.5) + [(3, 14, 0.2, 0.9)],
     0.04, 9, 3, {"tile_bits": 12, "reg_bits": 4, "no_merge": 1}),
    ("uncoupled-observed", spq.SPIN_C64, 16, [(1, 2, 0.0, 1.0), (5, 15, 0.0, 1.0)], 0.1, 100, 0,
     {"tile_bits": 12, "reg_bits": 4}),
    ("no-couplings", spq.SPIN_C64, 16, [], 0.1, 7, 4, {}),
    ("zero-steps", spq.SPIN_C128, 16, workloads.ladder(8), 0.1, 0, 0, {}),
    ("unfused", spq.SPIN_C64, 8, workloads.ladder(4), 0.1, 5, 0, {"schedule": 1}),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_plan_trace_realises_strang_product(case):
    name, prec, M, J, dt, steps, obs, opts = case
    o = spq.Options(**opts)
    trace = spq.spin_plan_trace(prec, M, J, dt, steps, obs, o)
    info = spq.spin_describe_plan(prec, M, J, dt, steps, obs, o)
    nfac = int((trace[:, 0] == 0).sum())
    assert nfac == info["factor_ops"]
    psi0 = oracle.random_phase_state(M, 0, 11)
    Pw, Nw, psiw = oracle.trotter_run(psi0, M, J, dt, steps, obs)
    Pt, psit = replay(trace, psi0, M, obs)
    assert sorted(Pt) == list(range(steps + 1))        # each observable exactly once
    assert np.abs(np.array([Pt[k] for k in range(steps + 1)]) - Pw).max() < 1e-11
    assert np.abs(psit - psiw).max() < 1e-11


PROFILE_CASES = [
    ("ladder10-resident", spq.SPIN_C64, 10, workloads.ladder(5), 0.05, 30, {}),
    ("star9-zz-resident", spq.SPIN_C128, 9, workloads.star(9, 3, a_over_b=-2.0), 0.07, 12, {}),
    ("ladder16-k12", spq.SPIN_C128, 16, workloads.ladder(8), 0.05, 12, {"tile_bits": 12}),
    ("ladder18-k14-long", spq.SPIN_C64, 18, workloads.ladder(9), 0.05, 70, {}),
    ("star15-k12", spq.SPIN_C64, 15, workloads.star(15, 8, a_over_b=1.0), 0.02, 5,
     {"tile_bits": 12, "reg_bits": 4}),
    ("chain17-c128-k13", spq.SPIN_C128, 17, workloads.chain(17), 0.1, 20, {}),
    ("no-couplings", spq.SPIN_C64, 16, [], 0.1, 3, {}),
    ("zero-steps", spq.SPIN_C64, 16, workloads.ladder(8), 0.1, 0, {}),
    ("unfused", spq.SPIN_C64, 8, workloads.ladder(4), 0.1, 4, {"schedule": 1}),
]


@pytest.mark.parametrize("case", PROFILE_CASES, ids=[c[0] for c in PROFILE_CASES])
def test_profile_plan_trace_observes_every_site_once(case):
    """The all-site profile's plan: every (step, site) observable appears
    exactly once, at a point of the op order where it equals the oracle's
    profile, and the factors still realise the Strang product."""
    name, prec, M, J, dt, steps, opts = case
    o = spq.Options(**opts)
    trace = spq.spin_plan_trace(prec, M, J, dt, steps, spq.SPIN_ALL_SITES, o)
    info = spq.spin_describe_plan(prec, M, J, dt, steps, spq.SPIN_ALL_SITES, o)
    assert int((trace[:, 0] == 0).sum()) == info["factor_ops"]
    psi0 = oracle.random_phase_state(M, 0, 3)
    Pw, _, psiw = oracle.trotter_profile(psi0, M, J, dt, steps)
    psi = psi0.copy()
    seen = {}
    for kind, a, b, A, B in trace:
        if kind == 1:
            key = (int(a), int(b))
            assert key not in seen, key
            seen[key] = oracle.local_polarization(psi, M, int(b))
        else:
            oracle.apply_factor(psi, M, int(a), int(b), A, B, 1.0)
    assert sorted(seen) == [(k, s) for k in range(steps + 1) for s in range(M)]
    got = np.array([[seen[(k, s)] for s in range(M)] for k in range(steps + 1)])
    assert np.abs(got - Pw).max() < 1e-11
    assert np.abs(psi - psiw).max() < 1e-11


def test_profile_plan_of_long_ladder_stays_fused():
    J = workloads.ladder(15)
    info = spq.spin_describe_plan(spq.SPIN_C64, 30, J, 0.05, 200, spq.SPIN_ALL_SITES)
    base = spq.spin_describe_plan(spq.SPIN_C64, 30, J, 0.05, 200, 0)
    assert info["path"] == 2
    # Observing every site between steps blocks only the merges across step
    # boundaries: at most one factor per coupling and step more.
    assert base["factor_ops"] < info["factor_ops"] <= base["factor_ops"] + 200 * len(J)
    # 30 per-site observables per step ride in the passes that hold their
    # sites (up to 64 per pass): the passes beyond the one-site plan's come
    # from the step-boundary merges the profile forgoes (about a fifth more
    # factors per step on this ladder).
    assert info["passes_per_step"] < 1.35 * base["passes_per_step"]
    with pytest.raises(spq.SpinError) as e:
        spq.spin_describe_plan(spq.SPIN_C64, 18, workloads.ladder(9), 0.05, 10, spq.SPIN_ALL_SITES,
                               spq.Options(engine=1))
    assert e.value.code == spq.SPIN_EUNSUPPORTED


def test_long_ladder_plan_is_periodic_and_fused():
    J = workloads.ladder(15)
    info = spq.spin_describe_plan(spq.SPIN_C64, 30, J, 0.05, 1000, 0)
    assert info["path"] == 2 and info["period_steps"] >= 1
    assert info["passes_per_step"] < 4.0          # versus 86 factors per step unfused
    info128 = spq.spin_describe_plan(spq.SPIN_C128, 30, J, 0.05, 1000, 0)
    assert info128["path"] == 2


def test_matrix_engine_option_checks():
    """The matrix engine exists for complex64 tiles of 2^14 with 32 registers
    per lane and whole-tile exchanges; other requests are refused on the
    host, and the plan (and so the op trace) is the butterfly plan's with
    whole-tile exchanges."""
    J = workloads.ladder(9)
    o = spq.Options(engine=1)
    info = spq.spin_describe_plan(spq.SPIN_C64, 18, J, 0.05, 10, 0, o)
    assert info["engine"] == 1 and info["reg_bits"] == 5 and info["tile_bits"] == 14
    assert info["exchange"] == 1
    t1 = spq.spin_plan_trace(spq.SPIN_C64, 18, J, 0.05, 10, 0, o)
    t0 = spq.spin_plan_trace(spq.SPIN_C64, 18, J, 0.05, 10, 0, spq.Options(exchange=1))
    assert np.array_equal(t0, t1)
    with pytest.raises(spq.SpinError) as e:
        spq.spin_describe_plan(spq.SPIN_C64, 18, J, 0.05, 10, 0, spq.Options(engine=1, exchange=2))
    assert e.value.code == spq.SPIN_EUNSUPPORTED
    with pytest.raises(spq.SpinError) as e:
        spq.spin_describe_plan(spq.SPIN_C64, 18, J, 0.05, 10, 0, spq.Options(exchange=3))
    assert e.value.code == spq.SPIN_EINVAL
    for prec, kw, code in [(spq.SPIN_C128, {}, spq.SPIN_EUNSUPPORTED),
                           (spq.SPIN_C64, {"tile_bits": 13}, spq.SPIN_EUNSUPPORTED),
                           (spq.SPIN_C64, {"reg_bits": 4}, spq.SPIN_EUNSUPPORTED)]:
        with pytest.raises(spq.SpinError) as e:
            spq.spin_describe_plan(prec, 18, J, 0.05, 10, 0, spq.Options(engine=1, **kw))
        assert e.value.code == code
    with pytest.raises(spq.SpinError) as e:
        spq.spin_describe_plan(spq.SPIN_C64, 18, J, 0.05, 10, 0, spq.Options(engine=2))
    assert e.value.code == spq.SPIN_EINVAL


def test_batch_rejects_bad_init_and_basis_index():
    """Argument errors of the batched call are found on the host before any
    device work (the state pointer is never dereferenced)."""
    lib = spq.load_library()
    arr, K = spq._couplings([(0, 1, 0.0, 1.0)])
    pr = (spq.Problem * 1)()
    pr[0].psi = 16
    pr[0].M = 4
    pr[0].K = 1
    pr[0].observed_site = 0
    pr[0].P_dev = 16
    pr[0].seed = 16          # basis index 16 >= 2^4
    rc = lib.spin_trotter_evolve_batch(pr, 1, arr, K, spq.SPIN_C64, 0.1, 3, spq.SPIN_INIT_BASIS, None)
    assert rc == spq.SPIN_EINVAL and "basis index" in spq.spin_last_error()
    rc = lib.spin_trotter_evolve_batch(pr, 1, arr, K, spq.SPIN_C64, 0.1, 3, 7, None)
    assert rc == spq.SPIN_EINVAL and "init" in spq.spin_last_error()


ENSEMBLE_BAD = [
    # (changes to the valid call, fragment of the message)
    ({"prec": 9}, "prec"),
    ({"M": 0}, "M = 0"),
    ({"polarized": 4}, "polarized_site"),
    ({"observed": -1}, "observed_site"),
    ({"n_members": 0}, "n_members"),
    ({"first": 1, "n_members": 8}, "member range"),
    ({"first": -1}, "member range"),
    ({"work_amps": 15}, "fewer than 2^M"),
    ({"work": 0}, "psi is NULL"),
    ({"work": 24}, "aligned"),
    ({"P": None}, "P_dev"),
    ({"n_steps": -1}, "n_steps"),
    ({"dt": float("nan")}, "dt"),
    ({"J": [(0, 4, 0.0, 1.0)]}, "site out of range"),
]


@pytest.mark.parametrize("change,frag", ENSEMBLE_BAD, ids=[f for _, f in ENSEMBLE_BAD])
def test_ensemble_argument_checks(change, frag):
    """spin_ensemble_evolve finds argument errors on the host before any
    device work (fake device pointers are never dereferenced)."""
    lib = spq.load_library()
    a = {"prec": spq.SPIN_C64, "M": 4, "J": [(0, 1, 0.0, 1.0), (1, 2, 0.0, 1.0)], "dt": 0.1,
         "n_steps": 3, "polarized": 0, "observed": 0, "first": 0, "n_members": 8, "work": 16,
         "work_amps": 64, "P": 32}
    a.update(change)
    arr, K = spq._couplings(a["J"])
    rc = lib.spin_ensemble_evolve(a["prec"], a["M"], arr, K, a["dt"], a["n_steps"], a["polarized"],
                                  a["observed"], a["first"], a["n_members"], a["work"], a["work_amps"],
                                  a["P"], None, None, None)
    assert rc == spq.SPIN_EINVAL and frag in spq.spin_last_error()


@pytest.mark.parametrize("seed", range(6))
def test_random_graphs_plan_and_encode(seed):
    """Random coupling graphs, sizes, shapes and step counts: the host-only
    description plans and encodes the tables exactly as the evolve call
    would, and must succeed (single site and all-site profile)."""
    rng = np.random.default_rng(seed)
    for _ in range(4):
        prec = [spq.SPIN_C64, spq.SPIN_C128][int(rng.integers(2))]
        M = int(rng.integers(2, 23))
        K = int(rng.integers(0, 3 * M))
        J = []
        for _ in range(K):
            i, j = (int(x) for x in rng.integers(0, M, size=2))
            if i != j:
                a = float(rng.uniform(-1, 1)) if rng.integers(3) == 0 else 0.0
                J.append((i, j, a, float(rng.uniform(-2, 2))))
        steps = int(rng.integers(0, 40))
        opts = {}
        if M > 14 and rng.integers(2):
            opts = {"tile_bits": 12, "reg_bits": 4}
        o = spq.Options(**opts)
        for obs in (int(rng.integers(M)), spq.SPIN_ALL_SITES):
            spq.spin_describe_plan(prec, M, J, 0.05, steps, obs, o)


def test_profile_plan_encodes_with_many_steps_per_pass():
    """One bond between the end sites: a profile pass spans many steps; its
    norm slots must stay within the pass's capacity (regression)."""
    for prec, M, steps in [(spq.SPIN_C64, 28, 4), (spq.SPIN_C128, 24, 50), (spq.SPIN_C64, 34, 4)]:
        info = spq.spin_describe_plan(prec, M, [(0, M - 1, 0.2, 0.9)], 0.1, steps, spq.SPIN_ALL_SITES)
        assert info["path"] == 2


# ------------------------------------------------------------------ exchanges
_XCHECK = None


def _exchange_check_binary(tmp_path_factory):
    """Builds tests/host_checks/exchange_check.cpp against the planner."""
    global _XCHECK
    if _XCHECK is None:
        out = str(tmp_path_factory.mktemp("xcheck") / "exchange_check")
        subprocess.check_call(["g++", "-O2", "-std=c++17",
                               os.path.join(ROOT, "tests", "host_checks", "exchange_check.cpp"),
                               os.path.join(ROOT, "paper_0710_3747_amd", "csrc", "planner.cpp"),
                               "-o", out])
        _XCHECK = out
    return _XCHECK


def _run_exchange_check(binary, M, J, prec, k, r, c, steps, obs=0, plant=0, half=0):
    inp = f"{M} {prec} {k} {r} {c} {steps} {obs} {plant} {half}\n" + "".join(
        f"{i} {j} {a!r} {b!r}\n" for i, j, a, b in J)
    p = subprocess.run([binary], input=inp, capture_output=True, text=True, timeout=600)
    return p.returncode, p.stdout


EXCHANGE_CASES = [
    # name, M, couplings, prec, k, r, c, steps, half-tile exchanges
    ("ladder2x15-c64-k14r5c4-half", 30, workloads.ladder(15), 1, 14, 5, 4, 1000, 1),
    # 2-stage passes whose only exchange stays in each wave (their first
    # exchange must carry the workgroup barrier)
    ("ladder2x15-c64-k14r5c5-half-3steps", 30, workloads.ladder(15), 1, 14, 5, 5, 3, 1),
    ("ladder2x15-c64-k14r5c4", 30, workloads.ladder(15), 1, 14, 5, 4, 100, 0),
    ("ladder2x15-c64-k14r5c6", 30, workloads.ladder(15), 1, 14, 5, 6, 100, 0),
    ("ladder2x15-c64-k14r6c4-half", 30, workloads.ladder(15), 1, 14, 6, 4, 100, 1),
    ("ladder2x15-c64-k14r4c4", 30, workloads.ladder(15), 1, 14, 4, 4, 100, 0),
    ("ladder2x15-c128-k13r4c4-half", 30, workloads.ladder(15), 2, 13, 4, 4, 100, 1),
    ("ladder2x15-c128-k13r5c4-half", 30, workloads.ladder(15), 2, 13, 5, 4, 100, 1),
    ("ladder2x15-c128-k14r5c4-half", 30, workloads.ladder(15), 2, 14, 5, 4, 100, 1),
    ("star28-c64-k14r5c6-half", 28, workloads.star(28, 33), 1, 14, 5, 6, 12, 1),
    ("star28-blocks-c64-k14r6c4-half", 28, workloads.star_m28(), 1, 14, 6, 4, 12, 1),
    ("star20-c64-k14r5c4", 20, workloads.star(20, 2000), 1, 14, 5, 4, 60, 0),
    ("ladder2x9-c128-k12r3c4", 18, workloads.ladder(9), 2, 12, 3, 4, 30, 0),
]


@pytest.mark.parametrize("case", EXCHANGE_CASES, ids=[c[0] for c in EXCHANGE_CASES])
def test_wave_local_exchanges_stay_in_their_wave(case, tmp_path_factory):
    """Every stage exchange the tables mark as wave-local (no workgroup
    barrier) moves amplitudes only within each wave, tile boundaries
    without a barrier keep every wave's LDS slots, and passes with no
    barrier at all store exactly the offsets each wave loaded -- by
    emulating the kernel's LDS and global address arithmetic on the host.
    Half-tile passes also keep their split position on the top register bit
    with no LDS image, and map each half one-to-one onto the buffer."""
    name, M, J, prec, k, r, c, steps, half = case
    rc, out = _run_exchange_check(_exchange_check_binary(tmp_path_factory), M, J, prec, k, r, c, steps,
                                  half=half)
    assert rc == 0, out
    assert "failures 0" in out


def test_exchange_check_reports_a_planted_cross_wave_exchange(tmp_path_factory):
    """The same check reports a failure when every exchange is (wrongly)
    marked wave-local."""
    rc, out = _run_exchange_check(_exchange_check_binary(tmp_path_factory), 30, workloads.ladder(15), 1,
                                  14, 5, 4, 40, plant=1)
    assert rc == 1 and "moves amplitudes between waves" in out


def test_describe_counts_stage_exchanges():
    """spin_plan_info.exchanges: the state held by one workgroup does one LDS
    round trip per stage (prologue once, the step's stages every step); a
    tiled plan does one per register stage after the first of each launch."""
    J = workloads.ladder(5)
    d0 = spq.spin_describe_plan(spq.SPIN_C64, 10, J, 0.05, 0, 0)
    d7 = spq.spin_describe_plan(spq.SPIN_C64, 10, J, 0.05, 7, 0)
    assert d0["path"] == 1 and d0["exchanges"] > 0
    assert (d7["exchanges"] - d0["exchanges"]) % 7 == 0 and d7["exchanges"] > d0["exchanges"]
    t = spq.spin_describe_plan(spq.SPIN_C64, 18, workloads.ladder(9), 0.05, 40, 0)
    assert t["path"] == 2
    assert 0 < t["exchanges"] < t["launches"] * 64
    assert t["exchanges"] >= t["stages_total"] - t["templates"]
