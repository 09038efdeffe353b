"""Python binding of the MI355X random-phase spin-dynamics library.

Thin ctypes layer over the C ABI declared in ``include/spin.h`` (same entry
point names).  It only marshals arguments: every step of the path runs in
the library's HIP kernels.  PyTorch supplies device memory and streams.

The library must be built first (``python -m paper_0710_3747_amd.build``);
every call raises ``RuntimeError`` when ``libspinqp.so`` is missing -- there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

import numpy as np

__all__ = [
    "SPIN_C64", "SPIN_C128", "SpinError", "library_path", "load_library",
    "spin_init_random_phase", "spin_init_product", "spin_trotter_evolve", "spin_trotter_evolve_ex",
    "spin_trotter_evolve_profile", "spin_trotter_evolve_noalloc", "SPIN_ALL_SITES",
    "spin_local_polarization", "spin_local_polarization_ex", "spin_trotter_evolve_batch",
    "spin_batch_status", "spin_ensemble_evolve", "spin_prepare_plan", "spin_describe_plan",
    "spin_plan_trace", "spin_last_error", "spin_release_caches", "spin_version",
    "Options", "Problem",
]

SPIN_OK, SPIN_EINVAL, SPIN_ENOMEM, SPIN_EHIP, SPIN_EUNSUPPORTED, SPIN_ENOTFOUND = 0, -1, -2, -3, -4, -5
SPIN_C64, SPIN_C128 = 1, 2
SPIN_INIT_NONE, SPIN_INIT_RANDOM_PHASE, SPIN_INIT_BASIS, SPIN_INIT_PRODUCT = 0, 1, 2, 3
SPIN_ALL_SITES = -1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "libspinqp.so")
_lib = None


class SpinError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"spin status {code}: {msg}")
        self.code = code


class _Coupling(ctypes.Structure):
    _fields_ = [("i", ctypes.c_int32), ("j", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double)]


class Options(ctypes.Structure):
    """``spin_options``; zero fields mean defaults."""
    _fields_ = [("schedule", ctypes.c_int32), ("tile_bits", ctypes.c_int32),
                ("reg_bits", ctypes.c_int32), ("coalesce_bits", ctypes.c_int32),
                ("engine", ctypes.c_int32), ("no_merge", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("exchange", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 8)]


class TuneResult(ctypes.Structure):
    """``spin_tune_result``."""
    _fields_ = [("opt", Options), ("ms_per_step", ctypes.c_double),
                ("trial_ms_per_step", ctypes.c_double),
                ("passes_per_step", ctypes.c_double), ("status", ctypes.c_int32),
                ("reserved_", ctypes.c_int32)]


class Problem(ctypes.Structure):
    """``spin_problem``."""
    _fields_ = [("psi", ctypes.c_void_p), ("M", ctypes.c_int32), ("K", ctypes.c_int32),
                ("coupling_offset", ctypes.c_int64), ("polarized_site", ctypes.c_int32),
                ("observed_site", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("P_dev", ctypes.c_void_p), ("N_dev", ctypes.c_void_p)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("tile_bits", ctypes.c_int32),
                ("reg_bits", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("coalesce_bits", ctypes.c_int32), ("templates", ctypes.c_int32),
                ("period_steps", ctypes.c_int32), ("period_passes", ctypes.c_int32),
                ("stages_total", ctypes.c_int32), ("engine", ctypes.c_int32),
                ("exchange", ctypes.c_int32), ("reserved_", ctypes.c_int32),
                ("launches", ctypes.c_int64), ("factor_ops", ctypes.c_int64),
                ("passes_per_step", ctypes.c_double), ("exchanges", ctypes.c_int64)]


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Loads libspinqp.so (raises RuntimeError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                           "`python -m paper_0710_3747_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                              ctypes.c_uint64, ctypes.c_double)
    cp = ctypes.POINTER(_Coupling)
    op = ctypes.POINTER(Options)
    lib.spin_init_random_phase.argtypes = [vp, i32, i32, i32, u64, vp]
    lib.spin_init_product.argtypes = [vp, i32, i32, i32, u64, vp]
    lib.spin_trotter_evolve.argtypes = [vp, i32, i32, cp, i32, dbl, i64, i32, vp, vp, vp]
    lib.spin_trotter_evolve_ex.argtypes = [vp, i32, i32, cp, i32, dbl, i64, i32, vp, vp, op, vp]
    lib.spin_trotter_evolve_profile.argtypes = [vp, i32, i32, cp, i32, dbl, i64, vp, vp, op, vp]
    lib.spin_trotter_evolve_noalloc.argtypes = [vp, i32, i32, cp, i32, dbl, i64, i32, vp, vp, op, vp]
    lib.spin_local_polarization.argtypes = [vp, i32, i32, i32, vp, vp]
    lib.spin_local_polarization_ex.argtypes = [vp, i32, i32, i32, vp, vp, vp]
    lib.spin_batch_status.argtypes = [vp]
    lib.spin_trotter_evolve_batch.argtypes = [ctypes.POINTER(Problem), i32, cp, i64, i32, dbl,
                                              i64, i32, vp]
    lib.spin_ensemble_evolve.argtypes = [i32, i32, cp, i32, dbl, i64, i32, i32, i64, i64, vp, i64,
                                         vp, vp, op, vp]
    lib.spin_prepare_plan.argtypes = [i32, i32, cp, i32, dbl, i64, i32, op]
    lib.spin_autotune.argtypes = [i32, i32, cp, i32, dbl, i32, i64, ctypes.c_char_p, op,
                                  ctypes.POINTER(TuneResult), i32, ctypes.POINTER(ctypes.c_int32), vp]
    lib.spin_tuned_options.argtypes = [i32, i32, cp, i32, dbl, i32, ctypes.c_char_p, op]
    lib.spin_describe_plan.argtypes = [i32, i32, cp, i32, dbl, i64, i32, op,
                                       ctypes.POINTER(_PlanInfo)]
    lib.spin_plan_trace.argtypes = [i32, i32, cp, i32, dbl, i64, i32, op,
                                    ctypes.POINTER(ctypes.c_double), i64,
                                    ctypes.POINTER(ctypes.c_int64)]
    lib.spin_last_error.restype = ctypes.c_char_p
    lib.spin_version.restype = ctypes.c_char_p
    lib.spin_release_caches.restype = None
    for name in ("spin_init_random_phase", "spin_init_product", "spin_trotter_evolve",
                 "spin_trotter_evolve_ex", "spin_trotter_evolve_noalloc",
                 "spin_trotter_evolve_profile",
                 "spin_local_polarization", "spin_local_polarization_ex",
                 "spin_trotter_evolve_batch", "spin_batch_status", "spin_ensemble_evolve",
                 "spin_prepare_plan",
                 "spin_describe_plan", "spin_plan_trace", "spin_autotune", "spin_tuned_options"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def spin_last_error() -> str:
    return load_library().spin_last_error().decode()


def spin_version() -> str:
    return load_library().spin_version().decode()


def spin_release_caches() -> None:
    load_library().spin_release_caches()


def _check(rc: int) -> None:
    if rc != SPIN_OK:
        raise SpinError(rc, spin_last_error())


def _couplings(J: Iterable[Sequence[float]]):
    J = list(J)
    arr = (_Coupling * max(1, len(J)))()
    for n, c in enumerate(J):
        arr[n].i, arr[n].j, arr[n].a, arr[n].b = int(c[0]), int(c[1]), float(c[2]), float(c[3])
    return arr, len(J)


def _prec_of(psi) -> int:
    import torch
    if psi.dtype == torch.complex64:
        return SPIN_C64
    if psi.dtype == torch.complex128:
        return SPIN_C128
    raise TypeError("psi must be complex64 or complex128")


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _state(psi, M: int):
    if not psi.is_cuda or not psi.is_contiguous():
        raise ValueError("psi must be a contiguous device tensor")
    if psi.numel() != 2 ** M:
        raise ValueError(f"psi holds {psi.numel()} amplitudes, 2^M = {2 ** M}")
    return ctypes.c_void_p(psi.data_ptr()), _prec_of(psi)


def _f64(t, n: int, name: str):
    import torch
    if t is None:
        return None
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() < n:
        raise ValueError(f"{name} must be a contiguous float64 device tensor of >= {n} entries")
    return ctypes.c_void_p(t.data_ptr())


def spin_init_random_phase(psi, M: int, polarized_site: int, seed: int, stream=None) -> None:
    """Writes the random-phase state into ``psi`` (see include/spin.h)."""
    lib = load_library()
    p, prec = _state(psi, M)
    _check(lib.spin_init_random_phase(p, prec, M, polarized_site, seed & (2 ** 64 - 1),
                                      _stream(stream)))


def spin_init_product(psi, M: int, polarized_site: int, seed: int, stream=None) -> None:
    """Writes the product state of M-1 random phases into ``psi`` (see include/spin.h)."""
    lib = load_library()
    p, prec = _state(psi, M)
    _check(lib.spin_init_product(p, prec, M, polarized_site, seed & (2 ** 64 - 1), _stream(stream)))


def spin_trotter_evolve_ex(psi, M: int, couplings, dt: float, n_steps: int, observed_site: int,
                           P, N=None, options: Optional[Options] = None, stream=None) -> None:
    lib = load_library()
    p, prec = _state(psi, M)
    arr, K = _couplings(couplings)
    _check(lib.spin_trotter_evolve_ex(p, prec, M, arr, K, float(dt), int(n_steps), observed_site,
                                      _f64(P, n_steps + 1, "P"), _f64(N, n_steps + 1, "N"),
                                      ctypes.byref(options) if options is not None else None,
                                      _stream(stream)))


def spin_trotter_evolve_noalloc(psi, M: int, couplings, dt: float, n_steps: int, observed_site: int,
                                P, N=None, options: Optional[Options] = None, stream=None) -> None:
    """spin_trotter_evolve_ex without device allocation (plan prepared first
    with spin_prepare_plan; see include/spin.h)."""
    lib = load_library()
    p, prec = _state(psi, M)
    arr, K = _couplings(couplings)
    _check(lib.spin_trotter_evolve_noalloc(p, prec, M, arr, K, float(dt), int(n_steps), observed_site,
                                           _f64(P, n_steps + 1, "P"), _f64(N, n_steps + 1, "N"),
                                           ctypes.byref(options) if options is not None else None,
                                           _stream(stream)))


def spin_trotter_evolve(psi, M: int, couplings, dt: float, n_steps: int, observed_site: int,
                        P, N=None, stream=None) -> None:
    """n_steps symmetric Trotter steps of ``psi`` in place; P[k], N[k] (FP64)."""
    spin_trotter_evolve_ex(psi, M, couplings, dt, n_steps, observed_site, P, N, None, stream)


def spin_trotter_evolve_profile(psi, M: int, couplings, dt: float, n_steps: int, Pall, N=None,
                                options: Optional[Options] = None, stream=None) -> None:
    """n_steps steps of ``psi`` in place with every site's polarisation after
    every step: Pall[k*M + n'] (FP64, (n_steps+1)*M entries), N[k]."""
    lib = load_library()
    p, prec = _state(psi, M)
    arr, K = _couplings(couplings)
    _check(lib.spin_trotter_evolve_profile(p, prec, M, arr, K, float(dt), int(n_steps),
                                           _f64(Pall, (n_steps + 1) * M, "Pall"),
                                           _f64(N, n_steps + 1, "N"),
                                           ctypes.byref(options) if options is not None else None,
                                           _stream(stream)))


def spin_local_polarization(psi, M: int, site: int, P, stream=None) -> None:
    """P[0] = polarisation of ``site`` in the state as it is (FP64 device tensor)."""
    lib = load_library()
    p, prec = _state(psi, M)
    _check(lib.spin_local_polarization(p, prec, M, site, _f64(P, 1, "P"), _stream(stream)))


def spin_local_polarization_ex(psi, M: int, site: int, P, N=None, stream=None) -> None:
    """P[0] = polarisation of ``site``, N[0] = norm (if N is given)."""
    lib = load_library()
    p, prec = _state(psi, M)
    _check(lib.spin_local_polarization_ex(p, prec, M, site, _f64(P, 1, "P"), _f64(N, 1, "N"),
                                          _stream(stream)))


def spin_batch_status(stream=None) -> int:
    """Synchronises the stream; 0 if no batched launch timed out at a gang
    barrier since the last query, else the error status (message in
    spin_last_error())."""
    return int(load_library().spin_batch_status(_stream(stream)))


def spin_trotter_evolve_batch(problems: Sequence[dict], prec: int, dt: float, n_steps: int,
                              init_random_phase: bool = True, stream=None,
                              init: Optional[int] = None) -> None:
    """Evolves independent problems in one launch (asynchronous on the
    stream; spin_batch_status() reports gang-barrier time-outs).

    Each problem is a dict with keys psi (device tensor), M, couplings,
    observed_site, P, optional N, polarized_site and seed.  `init` (one of
    SPIN_INIT_*) overrides init_random_phase; with SPIN_INIT_BASIS the seed
    is the basis index of the problem's initial state.
    """
    if init is None:
        init = SPIN_INIT_RANDOM_PHASE if init_random_phase else SPIN_INIT_NONE
    lib = load_library()
    allJ = []
    arr = (Problem * max(1, len(problems)))()
    for n, pr in enumerate(problems):
        psi = pr["psi"]
        ptr, pp = _state(psi, pr["M"])
        if pp != prec:
            raise ValueError("problem precision differs from prec")
        arr[n].psi = ptr.value
        arr[n].M = pr["M"]
        arr[n].K = len(pr["couplings"])
        arr[n].coupling_offset = len(allJ)
        allJ.extend(pr["couplings"])
        arr[n].polarized_site = pr.get("polarized_site", 0)
        arr[n].observed_site = pr["observed_site"]
        arr[n].seed = pr.get("seed", 0) & (2 ** 64 - 1)
        arr[n].P_dev = _f64(pr["P"], n_steps + 1, "P").value
        Nt = _f64(pr.get("N"), n_steps + 1, "N")
        arr[n].N_dev = Nt.value if Nt is not None else None
    carr, Ktot = _couplings(allJ)
    _check(lib.spin_trotter_evolve_batch(arr, len(problems), carr, Ktot, prec, float(dt),
                                         int(n_steps), int(init), _stream(stream)))


def spin_ensemble_evolve(work, M: int, couplings, dt: float, n_steps: int, polarized_site: int,
                         observed_site: int, P, N=None, first_member: int = 0,
                         n_members: Optional[int] = None, options: Optional[Options] = None,
                         stream=None) -> None:
    """Mean polarization over basis-state members of the ensemble of Eq. (1)
    (the whole ensemble by default); ``work`` is a contiguous complex64 or
    complex128 device tensor of at least 2^M amplitudes that the call
    overwrites (see include/spin.h)."""
    lib = load_library()
    if not work.is_cuda or not work.is_contiguous():
        raise ValueError("work must be a contiguous device tensor")
    prec = _prec_of(work)
    if n_members is None:
        n_members = 2 ** (M - 1) - first_member
    arr, K = _couplings(couplings)
    _check(lib.spin_ensemble_evolve(prec, M, arr, K, float(dt), int(n_steps), polarized_site,
                                    observed_site, int(first_member), int(n_members),
                                    ctypes.c_void_p(work.data_ptr()), work.numel(),
                                    _f64(P, n_steps + 1, "P"), _f64(N, n_steps + 1, "N"),
                                    ctypes.byref(options) if options is not None else None,
                                    _stream(stream)))


def spin_prepare_plan(prec: int, M: int, couplings, dt: float, n_steps: int, observed_site: int,
                      options: Optional[Options] = None) -> None:
    """Builds and caches on the current device the plan of the matching
    evolve call, so that call does no planning or table upload."""
    lib = load_library()
    arr, K = _couplings(couplings)
    _check(lib.spin_prepare_plan(prec, M, arr, K, float(dt), int(n_steps), observed_site,
                                 ctypes.byref(options) if options is not None else None))


def _opt_dict(o: "Options") -> dict:
    return {name: getattr(o, name) for name, _ in Options._fields_ if name != "reserved"}


def spin_autotune(prec: int, M: int, couplings, dt: float, observed_site: int,
                  trial_steps: int = 16, cache_path: Optional[str] = None, stream=None) -> dict:
    """Times the candidate launch shapes on a scratch state (blocking) and
    returns {"best": Options, "results": [dict per candidate]}."""
    lib = load_library()
    arr, K = _couplings(couplings)
    best = Options()
    res = (TuneResult * 16)()
    n = ctypes.c_int32(0)
    _check(lib.spin_autotune(prec, M, arr, K, float(dt), observed_site, int(trial_steps),
                             cache_path.encode() if cache_path else None, ctypes.byref(best),
                             res, 16, ctypes.byref(n), _stream(stream)))
    out = []
    for r in res[: min(n.value, 16)]:
        d = _opt_dict(r.opt)
        d.update(ms_per_step=r.ms_per_step, trial_ms_per_step=r.trial_ms_per_step,
                 passes_per_step=r.passes_per_step, status=r.status)
        out.append(d)
    return {"best": best, "results": out}


def spin_tuned_options(prec: int, M: int, couplings, dt: float, observed_site: int,
                       cache_path: Optional[str] = None) -> Optional["Options"]:
    """The stored autotuned options for these arguments, or None."""
    lib = load_library()
    arr, K = _couplings(couplings)
    best = Options()
    rc = lib.spin_tuned_options(prec, M, arr, K, float(dt), observed_site,
                                cache_path.encode() if cache_path else None, ctypes.byref(best))
    if rc == SPIN_ENOTFOUND:
        return None
    _check(rc)
    return best


def spin_describe_plan(prec: int, M: int, couplings, dt: float, n_steps: int, observed_site: int,
                       options: Optional[Options] = None) -> dict:
    """Host-only description of the plan the evolve call would run."""
    lib = load_library()
    arr, K = _couplings(couplings)
    info = _PlanInfo()
    _check(lib.spin_describe_plan(prec, M, arr, K, float(dt), int(n_steps), observed_site,
                                  ctypes.byref(options) if options is not None else None,
                                  ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in _PlanInfo._fields_ if name != "reserved_"}


def spin_plan_trace(prec: int, M: int, couplings, dt: float, n_steps: int, observed_site: int,
                    options: Optional[Options] = None) -> np.ndarray:
    """Executed op sequence as an (n, 5) array; see include/spin.h."""
    lib = load_library()
    arr, K = _couplings(couplings)
    n = ctypes.c_int64(0)
    optp = ctypes.byref(options) if options is not None else None
    _check(lib.spin_plan_trace(prec, M, arr, K, float(dt), int(n_steps), observed_site, optp,
                               None, 0, ctypes.byref(n)))
    buf = np.zeros((max(1, n.value), 5))
    _check(lib.spin_plan_trace(prec, M, arr, K, float(dt), int(n_steps), observed_site, optp,
                               buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n.value,
                               ctypes.byref(n)))
    return buf[: n.value]
