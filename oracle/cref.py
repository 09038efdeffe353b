"""ctypes wrapper of the plain C oracle loop (``trotter_ref.c``).

Test infrastructure only.  ``build()`` compiles the C file with gcc
(-O2 -fopenmp, IEEE arithmetic, no fast-math) into ``oracle/_build``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "liboracle_trotter.so")
_lib = None


def build(force: bool = True) -> str:
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    if force or not os.path.exists(_SO):
        subprocess.check_call([
            "gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
            os.path.join(_HERE, "trotter_ref.c"), "-o", _SO + ".tmp", "-lm"])
        os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_init_random_phase.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_uint64]
        lib.oracle_trotter_run.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, ip, dp, dp,
                                           ctypes.c_double, ctypes.c_int64, ctypes.c_int, dp, dp]
        lib.oracle_observe.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, dp]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def init_random_phase(M: int, n: int, seed: int) -> np.ndarray:
    psi = np.empty(2 ** M, dtype=np.complex128)
    _load().oracle_init_random_phase(_dp(psi.view(np.float64)), M, n, seed & (2 ** 64 - 1))
    return psi


def trotter_run(psi: np.ndarray, M: int, couplings, dt: float, n_steps: int, observed: int):
    """Evolve ``psi`` (complex128, modified in place); returns (P, N)."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.size == 2 ** M
    if not 0 <= observed < M:
        raise ValueError("observed site out of range")
    for c in couplings:     # the C loop indexes by site without checks
        if not (0 <= c[0] < M and 0 <= c[1] < M and c[0] != c[1]):
            raise ValueError(f"coupling {c} out of range for M={M}")
    K = len(couplings)
    ci = np.array([c[0] for c in couplings] or [0], dtype=np.int32)
    cj = np.array([c[1] for c in couplings] or [0], dtype=np.int32)
    ca = np.array([c[2] for c in couplings] or [0.0], dtype=np.float64)
    cb = np.array([c[3] for c in couplings] or [0.0], dtype=np.float64)
    P = np.empty(n_steps + 1)
    N = np.empty(n_steps + 1)
    ip = ctypes.POINTER(ctypes.c_int)
    _load().oracle_trotter_run(_dp(psi.view(np.float64)), M, K, ci.ctypes.data_as(ip),
                               cj.ctypes.data_as(ip), _dp(ca), _dp(cb), dt, n_steps,
                               observed, _dp(P), _dp(N))
    return P, N
