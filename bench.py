"""Benchmark of the random-phase Trotter path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--prec c64|c128|both] [--no-cpu-baseline]

Default workload: the 2 x 15 XY spin ladder (M = 30 sites, 43 couplings,
J = 1 on legs and rungs), dt = 0.05, site 0 polarised and observed, one
random-phase state (seed 5).  A bench "step" is one symmetric Trotter step
of the whole path (every pass of that step, with the observable fused).
Inputs are resident in HBM when the timed region starts; the timed region
is one spin_trotter_evolve call of K steps, bracketed by HIP events on the
stream the kernels run on.

value  = amplitude updates per second of the complex64 (FP32) path,
         2 K_c 2^M per Trotter step (each half-step factor counts once).
Also reported: the complex128 (FP64) path, the FP32-vs-FP64 error of P,
the pass kernel's roofline numbers and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "amplitude-updates/s + HBM GB/s per Trotter step at M=30, FP32 vs FP64 at stated err"
HBM_PEAK_GBS = 8000.0


def ladder_workload():
    import workloads
    L, dt, steps, seed = workloads.LADDER_CONFIGS["ladder_2x15"]
    return dict(name="ladder_2x15_xy", M=2 * L, J=workloads.ladder(L), dt=dt, steps=steps, seed=seed,
                observed=0, polarized=0)


def run_path(spq, torch, w, prec, steps, warmup, opts=None):
    """Returns dict with timing, P (host) and plan info for one precision."""
    M, J, dt = w["M"], w["J"], w["dt"]
    dtype = torch.complex64 if prec == spq.SPIN_C64 else torch.complex128
    psi = torch.empty(2 ** M, dtype=dtype, device="cuda")
    P = torch.empty(steps + 1, dtype=torch.float64, device="cuda")
    N = torch.empty(steps + 1, dtype=torch.float64, device="cuda")
    Pw = torch.empty(max(warmup, 0) + 1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    if warmup > 0:
        spq.spin_init_random_phase(psi, M, w["polarized"], w["seed"])
        spq.spin_trotter_evolve_ex(psi, M, J, dt, warmup, w["observed"], Pw, None, opts)
    # host planning and the table upload happen once per argument set, outside
    # the timed region (a cached plan is what repeated calls run)
    t_plan = time.perf_counter()
    spq.spin_prepare_plan(prec, M, J, dt, steps, w["observed"], opts)
    t_plan = time.perf_counter() - t_plan
    if opts is not None and opts.use_graph:
        # a graph is captured by the first call with these buffers: make that
        # call untimed, so the timed call replays it
        spq.spin_init_random_phase(psi, M, w["polarized"], w["seed"])
        spq.spin_trotter_evolve_ex(psi, M, J, dt, steps, w["observed"], P, N, opts)
    spq.spin_init_random_phase(psi, M, w["polarized"], w["seed"])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    spq.spin_trotter_evolve_ex(psi, M, J, dt, steps, w["observed"], P, N, opts)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    info = spq.spin_describe_plan(prec, M, J, dt, steps, w["observed"], opts)
    out = dict(ms_total=ms, wall_s=wall, P=P.cpu().numpy(), N=N.cpu().numpy(), info=info,
               plan_s=t_plan)
    del psi
    torch.cuda.empty_cache()
    return out


def run_profile(spq, torch, w, steps, opts=None):
    """All-site profile (every site's P after every step) on the complex64
    state: plan prepared outside the timed region, then one timed call."""
    M, J, dt = w["M"], w["J"], w["dt"]
    psi = torch.empty(2 ** M, dtype=torch.complex64, device="cuda")
    Pall = torch.empty((steps + 1) * M, dtype=torch.float64, device="cuda")
    N = torch.empty(steps + 1, dtype=torch.float64, device="cuda")
    spq.spin_init_random_phase(psi, M, w["polarized"], w["seed"])
    spq.spin_prepare_plan(spq.SPIN_C64, M, J, dt, steps, spq.SPIN_ALL_SITES, opts)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    spq.spin_trotter_evolve_profile(psi, M, J, dt, steps, Pall, N, opts)
    e1.record(stream)
    torch.cuda.synchronize()
    info = spq.spin_describe_plan(spq.SPIN_C64, M, J, dt, steps, spq.SPIN_ALL_SITES, opts)
    P = Pall.cpu().numpy().reshape(steps + 1, M)
    out = dict(ms_total=e0.elapsed_time(e1), P=P, N=N.cpu().numpy(), info=info)
    del psi
    torch.cuda.empty_cache()
    return out


def summarize(res, w, steps, prec_bytes):
    """Throughput and roofline figures of one timed run.

    The algorithmic bytes of one Trotter step are one sweep of the state,
    2S (read + write of 2^M amplitudes), however many pass launches the
    plan needs; a launch processes steps / launches of a step, so its
    algorithmic bytes are 2S * steps / launches and the achieved rate is
    2S * steps / timed seconds.  The per-launch sweep rate (2S per launch)
    is reported beside it as frac_per_pass."""
    M, K = w["M"], len(w["J"])
    amp_updates = 2 * K * 2 ** M * steps
    sec = res["ms_total"] / 1e3
    info = res["info"]
    launches = info["launches"]
    state_bytes = 2 ** M * prec_bytes
    sweep = 2 * state_bytes
    avg_launch_s = sec / launches
    alg_per_launch = sweep * steps / launches
    achieved = alg_per_launch / avg_launch_s / 1e9
    # every stage exchange writes and reads each amplitude once through LDS
    lds_bytes = info["exchanges"] * 2 * state_bytes
    return dict(value=amp_updates / sec, ms_per_step=res["ms_total"] / steps,
                passes_per_step=info["passes_per_step"], launches=launches,
                lds_bytes_per_step=lds_bytes / steps, lds_TBs=lds_bytes / sec / 1e12,
                avg_pass_ms=avg_launch_s * 1e3, achieved_gbs=achieved,
                alg_bytes_per_launch=alg_per_launch, alg_bytes_per_step=sweep,
                sweep_gbs_per_pass=sweep / avg_launch_s / 1e9,
                hbm_gbs_per_step=launches * sweep / sec / 1e9,
                one_sweep_frac=(sweep * steps / sec / 1e9) / HBM_PEAK_GBS)


def other_workload(name):
    import workloads
    if name in ("ladder_2x5", "ladder_2x12", "ladder_2x15"):
        L, dt, steps, seed = workloads.LADDER_CONFIGS[name]
        return dict(name=name + "_xy", M=2 * L, J=workloads.ladder(L), dt=dt, steps=steps, seed=seed,
                    observed=0, polarized=0)
    if name == "star_28":
        c = workloads.STAR_M28
        return dict(name="star_28_xy_blocks", M=c["M"], J=workloads.star_m28(),
                    dt=c["dt"], steps=c["n_steps"], seed=c["seed"], observed=0, polarized=0)
    raise ValueError(name)


# Non-packed FP32 VALU peak of the chip: 256 CUs x 4 SIMDs x 16 lanes x 2 flops
# (one FMA) x 2.4 GHz.  HIP code here is built without packed FP32.
VALU_F32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# VALU work of one amplitude update of the XY butterflies: a factor moves the
# 2^(M-2) anti-aligned pairs with a three-shear rotation of 6 FMAs per pair,
# i.e. 1.5 FMA = 3 flops per amplitude of the state.
FLOPS_PER_AMP_UPDATE = 3.0


def run_batch(spq, torch, prec=None, reps=2):
    """256 independent stars (M uniform in 14..20), 500 steps, one
    persistent launch (after one untimed call that plans and warms).
    Returns (summary, P of every problem as a host array)."""
    import numpy as np
    import workloads
    prec = spq.SPIN_C64 if prec is None else prec
    dtype = torch.complex64 if prec == spq.SPIN_C64 else torch.complex128
    cfg = workloads.BATCH_STARS
    spec = workloads.star_batch(cfg["n"], cfg["m_lo"], cfg["m_hi"], cfg["size_seed"],
                                cfg["coupling_seed0"], cfg["state_seed0"])
    steps, dt = cfg["n_steps"], cfg["dt"]
    probs = []
    for p in spec:
        probs.append(dict(psi=torch.empty(2 ** p["M"], dtype=dtype, device="cuda"),
                          M=p["M"], couplings=p["couplings"], observed_site=0, polarized_site=0,
                          seed=p["seed"], P=torch.zeros(steps + 1, dtype=torch.float64, device="cuda"),
                          N=None))
    spq.spin_trotter_evolve_batch(probs, prec, dt, steps, init_random_phase=True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        spq.spin_trotter_evolve_batch(probs, prec, dt, steps, init_random_phase=True)
    e1.record(stream)
    torch.cuda.synchronize()
    if spq.spin_batch_status() != 0:
        raise RuntimeError("batched stars: " + spq.spin_last_error())
    sec = e0.elapsed_time(e1) / 1e3 / reps
    upd = sum(2 * len(p["couplings"]) * 2 ** p["M"] * steps for p in spec)
    flops = FLOPS_PER_AMP_UPDATE * upd
    out = {"workload": "batch_256_stars_M14to20", "state": "complex64" if prec == spq.SPIN_C64
           else "complex128", "steps": steps, "seconds": sec,
           "amplitude_updates_per_s": upd / sec, "problems": len(spec),
           "amplitude_updates": upd,
           "state_bytes": sum((8 if prec == spq.SPIN_C64 else 16) * 2 ** p["M"] for p in spec)}
    if prec == spq.SPIN_C64:
        # LDS bytes of the stage exchanges, estimated from one problem of each
        # size planned on the single path at the batch's launch shape
        o = spq.Options(tile_bits=14, reg_bits=6, coalesce_bits=4)
        lds, seen = 0.0, {}
        for p in spec:
            if p["M"] not in seen:
                info = spq.spin_describe_plan(prec, p["M"], p["couplings"], dt, steps, 0, o)
                seen[p["M"]] = info["exchanges"] * 2 * 8 * 2 ** p["M"]
            lds += seen[p["M"]]
        out["roofline"] = {"bound": "alu", "achieved": flops / sec / 1e12,
                           "peak": VALU_F32_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": flops / sec / 1e12 / VALU_F32_PEAK_TFLOPS, "traffic": None,
                           "flops_per_amplitude_update": FLOPS_PER_AMP_UPDATE,
                           "lds_bytes_estimate": lds, "lds_TBs_estimate": lds / sec / 1e12,
                           "kernel": "k_batch"}
    return out, np.stack([p["P"].cpu().numpy() for p in probs])


def run_star(spq, torch, steps, warmup):
    """The all-to-all star M = 28 (378 couplings, block order) in both
    precisions, at the complex64 shape with 64 amplitudes per lane (k 14,
    r 6, c 4, half-tile exchanges) and the complex128 shape with tiles of
    2^14 (k 14, r 5, c 4; 10 instead of 18 passes per step)."""
    import numpy as np
    w = other_workload("star_28")
    o = spq.Options(tile_bits=14, reg_bits=6, coalesce_bits=4)
    o64 = spq.Options(tile_bits=14, reg_bits=5, coalesce_bits=4)
    r32 = run_path(spq, torch, w, spq.SPIN_C64, steps, warmup, o)
    r64 = run_path(spq, torch, w, spq.SPIN_C128, steps, warmup, o64)
    s32 = summarize(r32, w, steps, 8)
    s64 = summarize(r64, w, steps, 16)
    return {"workload": w["name"], "M": w["M"], "couplings": len(w["J"]), "dt": w["dt"],
            "steps": steps, "value": s32["value"], "unit": "amplitude-updates/s",
            "ms_per_step": s32["ms_per_step"], "passes_per_step": s32["passes_per_step"],
            "one_sweep_frac": s32["one_sweep_frac"],
            "shape": {k: r32["info"][k] for k in ("tile_bits", "reg_bits", "lanes", "coalesce_bits",
                                                  "exchange")},
            "fp64": {"value": s64["value"], "ms_per_step": s64["ms_per_step"],
                     "passes_per_step": s64["passes_per_step"]},
            "err_P_fp32_vs_fp64": float(np.abs(r32["P"] - r64["P"]).max())}


def run_ensemble(spq, torch, dt=0.05, draws=256, work_gib=32):
    """The method's own speed-up (Eq. (1) against Eq. (2)): the 2^(M-1)
    basis-state members of the ensemble evolved one by one on the GPU
    (spin_ensemble_evolve, member average on the device), against one
    random-phase state of the same ladder; at M = 14 also the members as
    one batched launch and the mean of independent phase draws (Eq. (4))."""
    import numpy as np
    import workloads
    out = []
    for L, steps in ((7, 100), (9, 50)):
        M = 2 * L
        J = workloads.ladder(L)
        D = 2 ** (M - 1)
        members_per_evolution = min(D, (work_gib << 30) // (8 * 2 ** M))
        work = torch.empty(members_per_evolution * 2 ** M, dtype=torch.complex64, device="cuda")
        Pe = torch.empty(steps + 1, dtype=torch.float64, device="cuda")
        t_ens = None
        for rep in range(2):      # the first call plans
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            spq.spin_ensemble_evolve(work, M, J, dt, steps, 0, 0, Pe)
            torch.cuda.synchronize()
            t_ens = time.perf_counter() - t0
        del work
        torch.cuda.empty_cache()
        Pbar = Pe.cpu().numpy()
        psi = torch.empty(2 ** M, dtype=torch.complex64, device="cuda")
        P1 = torch.empty(steps + 1, dtype=torch.float64, device="cuda")
        for rep in range(2):
            spq.spin_init_random_phase(psi, M, 0, 7)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            spq.spin_trotter_evolve(psi, M, J, dt, steps, 0, P1)
            torch.cuda.synchronize()
            t_one = time.perf_counter() - t0
        n_factors = 2 * len(J)
        r = {"workload": f"ladder_2x{L}_xy", "M": M, "steps": steps, "dt": dt,
             "ensemble_members": D, "members_per_evolution": members_per_evolution,
             "ensemble_seconds": t_ens,
             "ensemble_amplitude_updates_per_s": D * 2.0 ** M * n_factors * steps / t_ens,
             "one_random_phase_seconds": t_one,
             "ensemble_over_one_state": t_ens / t_one,
             "max_dP_one_state_vs_ensemble": float(np.abs(P1.cpu().numpy() - Pbar).max()),
             "bound_std_one_state": 2.0 * 2.0 ** (-(M - 1) / 2)}
        if L == 7:
            def batch(seeds, init):
                big = torch.empty(len(seeds), 2 ** M, dtype=torch.complex64, device="cuda")
                Pb = torch.zeros(len(seeds), steps + 1, dtype=torch.float64, device="cuda")
                probs = [dict(psi=big[i], M=M, couplings=J, observed_site=0, polarized_site=0,
                              seed=int(x), P=Pb[i]) for i, x in enumerate(seeds)]
                spq.spin_trotter_evolve_batch(probs, spq.SPIN_C64, dt, steps, init=init)   # plans
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                spq.spin_trotter_evolve_batch(probs, spq.SPIN_C64, dt, steps, init=init)
                torch.cuda.synchronize()
                sec = time.perf_counter() - t0
                if spq.spin_batch_status() != 0:
                    raise RuntimeError("ensemble batch: " + spq.spin_last_error())
                return sec, Pb.cpu().numpy()

            xs = [x for x in range(2 ** M) if not (x & 1)]
            t_b, P_b = batch(xs, spq.SPIN_INIT_BASIS)
            t_draws, P_draws = batch(list(range(draws)), spq.SPIN_INIT_RANDOM_PHASE)
            r.update({"batched_members_seconds": t_b,
                      "max_dP_batched_members_vs_ensemble": float(np.abs(P_b.mean(0) - Pbar).max()),
                      "phase_draws": draws, "phase_draws_seconds": t_draws,
                      "max_dP_mean_of_draws_vs_ensemble": float(np.abs(P_draws.mean(0) - Pbar).max())})
        out.append(r)
    return out


def shape_key(prec_name, info):
    return "%s_k%d_r%d_c%d_x%d" % (prec_name, info["tile_bits"], info["reg_bits"], info["coalesce_bits"],
                                   info.get("exchange", 1))


def measured_traffic(key):
    """HBM bytes per pass-kernel launch of launch shape `key` (shape_key) from
    the committed rocprofv3 counter summary, or None when that shape was not
    measured or the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_pass_ladder2x15_M30_traffic.json")
    src = os.path.join(ROOT, "paper_0710_3747_amd", "csrc")
    try:
        t = json.load(open(path))
        h = hashlib.sha256()
        for f in ("kernels.hip", "device_plan.hpp"):
            h.update(open(os.path.join(src, f), "rb").read())
        if h.hexdigest()[:16] != t["kernel_source_sha256_16"]:
            return None
        return t["shapes"][key]["traffic_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def cpu_model():
    """Host CPU model name (Linux /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, n_couplings=None, steps=2):
    """The plain C oracle on a bounded sample of the same workload: `steps`
    Strang steps (all couplings, 2K factor applications each, steps + 1
    observables) of the M = 30 state, complex128, all OpenMP threads
    (about 10 s on 16 threads)."""
    import numpy as np
    from oracle import cref
    cref.build(force=False)
    M = w["M"]
    psi = cref.init_random_phase(M, w["polarized"], w["seed"])
    J = w["J"] if n_couplings is None else w["J"][:n_couplings]
    t0 = time.perf_counter()
    cref.trotter_run(psi, M, J, w["dt"], steps, w["observed"])
    sec = time.perf_counter() - t0
    del psi
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    nfac = 2 * len(J) * steps
    return dict(value=nfac * 2 ** M / sec, unit="amplitude-updates/s", cores=threads, kind="oracle",
                sample=f"{steps} Strang steps ({nfac} factor applications of {len(J)} couplings, "
                       f"{steps + 1} observables) of the M={M} complex128 state; {sec:.2f} s",
                seconds=sec)


def cpu_single_core(w, M=26, n_couplings=20):
    """The same C oracle on one thread (a child process with
    OMP_NUM_THREADS=1): one Strang step of the first n_couplings couplings
    among sites below M on an M=26 state (1 GiB, beyond the host caches)."""
    import subprocess
    code = (
        "import json,sys,time\n"
        f"sys.path.insert(0,{ROOT!r})\n"
        "from oracle import cref\n"
        "cref.build(force=False)\n"
        f"J={[c for c in w['J'] if max(c[0], c[1]) < M][:n_couplings]!r}\n"
        f"psi=cref.init_random_phase({M},{w['polarized']},{w['seed']})\n"
        "t0=time.perf_counter()\n"
        f"cref.trotter_run(psi,{M},J,{w['dt']!r},1,{w['observed']})\n"
        "print(json.dumps({'seconds':time.perf_counter()-t0}))\n")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=600, check=True)
    sec = json.loads(out.stdout.strip().splitlines()[-1])["seconds"]
    nfac = 2 * n_couplings
    return dict(value=nfac * 2 ** M / sec, unit="amplitude-updates/s", cores=1, kind="oracle",
                sample=f"one Strang step of the first {n_couplings} couplings ({nfac} factor "
                       f"applications, 2 observables) of an M={M} complex128 state, one thread; "
                       f"{sec:.2f} s")


def copy_probe(torch, gib=4, reps=5):
    """Plain device-to-device copy of `gib` GiB (torch's copy kernel): the
    reference for the HBM byte counters and the achievable copy bandwidth."""
    n = gib * 2 ** 30 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * n * 4 / (ms / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "ms": ms, "copy_GBs": gbs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prec", default="both", choices=["c64", "c128", "both"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile-bits", type=int, default=0)
    ap.add_argument("--reg-bits", type=int, default=0)
    ap.add_argument("--coalesce-bits", type=int, default=0)
    ap.add_argument("--workload", default="ladder_2x15",
                    choices=["ladder_2x15", "ladder_2x12", "ladder_2x5", "star_28", "batch_stars",
                             "ensemble"])
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-stars extra")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default launch shape instead of the autotuner's choice")
    ap.add_argument("--engine-steps", type=int, default=100,
                    help="steps of the MFMA-matrix vs VALU-butterfly comparison (0 = skip)")
    ap.add_argument("--graph", action="store_true",
                    help="launch the timed path through a captured hipGraph (captured untimed)")
    ap.add_argument("--profile-steps", type=int, default=100,
                    help="steps of the all-site profile leg (0 = skip)")
    ap.add_argument("--star-steps", type=int, default=100,
                    help="steps of the M = 28 star leg, both precisions (0 = skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only time a plain device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the state would shard over the top address bits across GPUs; not built).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_0710_3747_amd as spq
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:
        print(json.dumps(copy_probe(torch)), flush=True)
        return
    spq.load_library()
    if args.workload == "ensemble":
        print(json.dumps(run_ensemble(spq, torch)), flush=True)
        return
    if args.workload == "batch_stars":
        print(json.dumps(run_batch(spq, torch)[0]), flush=True)
        return
    w = ladder_workload() if args.workload == "ladder_2x15" else other_workload(args.workload)
    steps, warmup = args.steps, args.warmup

    opts = None
    if args.tile_bits or args.reg_bits or args.coalesce_bits:
        opts = spq.Options(tile_bits=args.tile_bits, reg_bits=args.reg_bits,
                           coalesce_bits=args.coalesce_bits)
    res32 = res64 = None
    tuned = {}

    def shape_for(prec):
        # explicit shape flags win; otherwise the autotuner's choice (timed
        # trials before the timed region), unless disabled
        if opts is not None or args.no_autotune:
            return opts
        print(f"[bench] autotuning prec {prec}", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        out = spq.spin_autotune(prec, w["M"], w["J"], w["dt"], w["observed"], trial_steps=16)
        tuned["c64" if prec == spq.SPIN_C64 else "c128"] = {
            "seconds": time.perf_counter() - t0, "trial_steps": 16,
            "candidates": [{k: r[k] for k in ("tile_bits", "reg_bits", "coalesce_bits", "engine", "exchange",
                                               "ms_per_step", "trial_ms_per_step", "passes_per_step")}
                           for r in out["results"]],
            "chosen": {k: getattr(out["best"], k) for k in ("tile_bits", "reg_bits", "coalesce_bits", "engine",
                                                            "exchange")}}
        return out["best"]

    def with_graph(o):
        if not args.graph:
            return o
        g = spq.Options()
        if o is not None:
            ctypes.memmove(ctypes.addressof(g), ctypes.addressof(o), ctypes.sizeof(g))
        g.use_graph = 1
        return g

    if args.prec in ("c64", "both"):
        o = with_graph(shape_for(spq.SPIN_C64))
        print(f"[bench] complex64 path, {steps} steps", file=sys.stderr, flush=True)
        res32 = run_path(spq, torch, w, spq.SPIN_C64, steps, warmup, o)
    if args.prec in ("c128", "both"):
        o = with_graph(shape_for(spq.SPIN_C128))
        print(f"[bench] complex128 path, {steps} steps", file=sys.stderr, flush=True)
        res64 = run_path(spq, torch, w, spq.SPIN_C128, steps, warmup, o)

    head = res32 if res32 is not None else res64
    head_bytes = 8 if res32 is not None else 16
    s = summarize(head, w, steps, head_bytes)
    traffic = (measured_traffic(shape_key("c64" if res32 is not None else "c128", head["info"]))
               if args.workload == "ladder_2x15" else None)
    out = {
        "metric": METRIC,
        "value": s["value"],
        "unit": "amplitude-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": s["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if res32 is not None else "f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "M": w["M"], "couplings": len(w["J"]),
                   "factors_per_step": 2 * len(w["J"]), "dt": w["dt"], "seed": w["seed"],
                   "state": "complex64" if res32 is not None else "complex128",
                   "observable": "FP64 P and norm every step"},
        "roofline": {"bound": "hbm", "achieved": s["achieved_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": s["achieved_gbs"] / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, scaled)",
                     "traffic_per_step": traffic * s["launches"] / steps if traffic else None,
                     "alg_bytes_per_launch": s["alg_bytes_per_launch"],
                     "alg_bytes_per_step": s["alg_bytes_per_step"],
                     "frac_per_pass": s["sweep_gbs_per_pass"] / HBM_PEAK_GBS,
                     # LDS bytes of the stage exchanges (from the plan) and
                     # their rate over the timed region
                     "lds_bytes_per_step": s["lds_bytes_per_step"], "lds_TBs": s["lds_TBs"],
                     "kernel": "k_pass", "avg_launch_ms": s["avg_pass_ms"],
                     "launches": s["launches"],
                     # a state within the 256 MB Infinity Cache streams from
                     # there, not from HBM
                     "state_bytes": 2 ** w["M"] * head_bytes,
                     "cache_resident": 2 ** w["M"] * head_bytes <= 256 * 2 ** 20},
        "passes_per_step": s["passes_per_step"],
        "launch": "hipGraph replay" if args.graph else "stream",
        "plan_seconds": head["plan_s"],
        "shape": {k: head["info"][k] for k in ("tile_bits", "reg_bits", "lanes", "coalesce_bits", "exchange")},
        "hbm_gbs_per_step": s["hbm_gbs_per_step"],
        "one_sweep_frac": s["one_sweep_frac"],
    }
    if res32 is not None and res64 is not None:
        s64 = summarize(res64, w, steps, 16)
        import numpy as np
        out["fp64"] = {"value": s64["value"], "ms_per_step": s64["ms_per_step"],
                       "passes_per_step": s64["passes_per_step"],
                       "achieved_gbs": s64["achieved_gbs"],
                       "frac": s64["achieved_gbs"] / HBM_PEAK_GBS,
                       "frac_per_pass": s64["sweep_gbs_per_pass"] / HBM_PEAK_GBS}
        out["fp32_speedup_vs_fp64"] = s["value"] / s64["value"]
        out["err_P_fp32_vs_fp64"] = float(np.abs(res32["P"] - res64["P"]).max())
        out["norm_drift_fp32"] = float(np.abs(res32["N"] - 1).max())
        out["norm_drift_fp64"] = float(np.abs(res64["N"] - 1).max())
    if tuned:
        out["autotune"] = tuned
    if args.workload == "ladder_2x15":
        # second denominator: what a plain device copy reaches on this GPU
        # (torch's copy kernel, 4 GiB read + 4 GiB written), outside the timed region
        cp = copy_probe(torch)
        out["roofline"]["copy_GBs"] = cp["copy_GBs"]
        out["roofline"]["frac_of_copy"] = s["achieved_gbs"] / cp["copy_GBs"]
        out["roofline"]["frac_of_copy_per_pass"] = s["sweep_gbs_per_pass"] / cp["copy_GBs"]
    if args.workload == "ladder_2x15" and res32 is not None and args.engine_steps > 0:
        # stage arithmetic on FP32 MFMA (each stage's factors as one dense
        # 32 x 32 complex matrix) against the VALU butterflies, same shape
        import numpy as np
        n = min(args.engine_steps, steps)
        # both on whole-tile exchanges (the matrix engine's only form)
        base = dict(tile_bits=14, reg_bits=5, coalesce_bits=5, exchange=1)
        print(f"[bench] engine comparison, {n} steps", file=sys.stderr, flush=True)
        rb = run_path(spq, torch, w, spq.SPIN_C64, n, 2, spq.Options(**base))
        rm = run_path(spq, torch, w, spq.SPIN_C64, n, 2, spq.Options(engine=1, **base))
        cmp = {"steps": n, "shape": base,
               "butterfly_ms_per_step": rb["ms_total"] / n, "mfma_ms_per_step": rm["ms_total"] / n,
               "mfma_time_ratio": rm["ms_total"] / rb["ms_total"],
               "passes_per_step": rm["info"]["passes_per_step"],
               "max_dP_mfma_vs_butterfly": float(np.abs(rm["P"] - rb["P"]).max())}
        if res64 is not None:
            cmp["max_dP_mfma_vs_fp64"] = float(np.abs(rm["P"] - res64["P"][: n + 1]).max())
        out["engine_comparison"] = cmp
    if args.workload == "ladder_2x15" and res32 is not None and args.star_steps > 0:
        n = min(args.star_steps, steps)
        print(f"[bench] star M=28, {n} steps", file=sys.stderr, flush=True)
        out["star_28"] = run_star(spq, torch, n, 2)
    if args.workload == "ladder_2x15" and res32 is not None and args.profile_steps > 0:
        # every site's polarisation after every step, in the same passes
        import numpy as np
        n = min(args.profile_steps, steps)
        # the shape the headline ran with (explicit, autotuned, or default)
        o = opts if (opts is not None or args.no_autotune) else spq.spin_tuned_options(
            spq.SPIN_C64, w["M"], w["J"], w["dt"], w["observed"])
        print(f"[bench] all-site profile, {n} steps", file=sys.stderr, flush=True)
        rp = run_profile(spq, torch, w, n, o)
        rs = run_path(spq, torch, w, spq.SPIN_C64, n, 2, o)
        out["all_site_profile"] = {
            "steps": n, "sites": w["M"],
            "ms_per_step": rp["ms_total"] / n,
            "single_site_ms_per_step": rs["ms_total"] / n,
            "time_ratio": rp["ms_total"] / rs["ms_total"],
            "passes_per_step": rp["info"]["passes_per_step"],
            "max_dP_site0_vs_single_site": float(np.abs(rp["P"][:, w["observed"]] - rs["P"]).max()),
            "max_total_polarisation_drift": float(np.abs(rp["P"].sum(axis=1) - rp["P"][0].sum()).max())}
    if args.workload != "ladder_2x15":
        out["metric"] = "amplitude-updates/s per Trotter step (secondary workload)"
    elif not args.no_batch:
        import numpy as np
        print("[bench] batched stars", file=sys.stderr, flush=True)
        bs, P32 = run_batch(spq, torch)
        print("[bench] batched stars, complex128", file=sys.stderr, flush=True)
        bs64, P64 = run_batch(spq, torch, spq.SPIN_C128, reps=1)
        bs["fp64"] = {k: bs64[k] for k in ("seconds", "amplitude_updates_per_s", "state_bytes")}
        bs["err_P_fp32_vs_fp64"] = float(np.abs(P32 - P64).max())
        out["batch_stars"] = bs
        print("[bench] basis-state ensemble vs random phase", file=sys.stderr, flush=True)
        out["ensemble_vs_random_phase"] = run_ensemble(spq, torch)
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle sample", file=sys.stderr, flush=True)
        cb = cpu_baseline(w)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline"]["cpu_model"] = cpu_model()
        out["cpu_baseline_single_core"] = cpu_single_core(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
