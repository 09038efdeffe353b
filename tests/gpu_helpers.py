"""Shared helpers of the GPU tests: run the HIP path through the C ABI and
fetch results to the host.  (Not collected by pytest: no test_ prefix.)"""
import sys

import numpy as np

import paper_0710_3747_amd as spq


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def torch_dtype(prec):
    import torch
    return torch.complex64 if prec == spq.SPIN_C64 else torch.complex128


def gpu_state(prec, M, polarized=0, seed=1, psi0=None):
    import torch
    if psi0 is not None:
        return torch.from_numpy(np.ascontiguousarray(psi0)).to(torch_dtype(prec)).cuda()
    psi = torch.empty(2 ** M, dtype=torch_dtype(prec), device="cuda")
    spq.spin_init_random_phase(psi, M, polarized, seed)
    return psi


def gpu_evolve(prec, M, J, dt, steps, observed, polarized=0, seed=1, opts=None, psi=None,
               psi0=None, keep_state=True):
    """Returns (P, N, psi_numpy_or_None, psi_tensor)."""
    import torch
    if psi is None:
        psi = gpu_state(prec, M, polarized, seed, psi0)
    P = torch.full((steps + 1,), float("nan"), dtype=torch.float64, device="cuda")
    N = torch.full((steps + 1,), float("nan"), dtype=torch.float64, device="cuda")
    o = spq.Options(**opts) if opts else None
    spq.spin_trotter_evolve_ex(psi, M, J, dt, steps, observed, P, N, o)
    torch.cuda.synchronize()
    out = psi.cpu().numpy().astype(np.complex128) if keep_state else None
    return P.cpu().numpy(), N.cpu().numpy(), out, psi


# tolerances: P absolute (FP64 1e-10, FP32 1e-4); amplitudes relative to the largest
TOL_P = {spq.SPIN_C128: 1e-10, spq.SPIN_C64: 1e-4}
TOL_PSI = {spq.SPIN_C128: 1e-10, spq.SPIN_C64: 1e-4}


def assert_state_close(got, want, prec):
    scale = np.abs(want).max()
    err = np.abs(got - want).max() / scale
    assert err < TOL_PSI[prec], f"state rel err {err:.3e}"


def gpu_profile(prec, M, J, dt, steps, polarized=0, seed=1, opts=None, psi0=None,
                keep_state=True):
    """All-site profile through spin_trotter_evolve_profile.

    Returns (Pall (steps+1, M), N, psi_numpy or None)."""
    import torch
    psi = gpu_state(prec, M, polarized, seed, psi0)
    Pall = torch.full(((steps + 1) * M,), float("nan"), dtype=torch.float64, device="cuda")
    N = torch.full((steps + 1,), float("nan"), dtype=torch.float64, device="cuda")
    o = spq.Options(**opts) if opts else None
    spq.spin_trotter_evolve_profile(psi, M, J, dt, steps, Pall, N, o)
    torch.cuda.synchronize()
    out = psi.cpu().numpy().astype(np.complex128) if keep_state else None
    return Pall.cpu().numpy().reshape(steps + 1, M), N.cpu().numpy(), out
