"""The allocation-free evolve entry point (spin_trotter_evolve_noalloc),
through the C ABI, against spin_trotter_evolve_ex on the same inputs: two
calls in a row (the second on a smaller state), bit for bit, with no change
in the device's free memory across each call once the first call on the
device has looked up its array."""
import ctypes

import numpy as np
import pytest

import workloads
import paper_0710_3747_amd as spq
from gpu_helpers import note, torch_dtype

pytestmark = pytest.mark.gpu


def _c_args(J):
    arr = (spq._Coupling * max(1, len(J)))()
    for n, c in enumerate(J):
        arr[n].i, arr[n].j, arr[n].a, arr[n].b = int(c[0]), int(c[1]), float(c[2]), float(c[3])
    return arr, len(J)


def _run(lib, fn, psi, prec, M, J, dt, steps, obs, P, N, opt, torch):
    arr, K = _c_args(J)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    optp = ctypes.byref(opt) if opt is not None else None
    return getattr(lib, fn)(ctypes.c_void_p(psi.data_ptr()), prec, M, arr, K, float(dt), int(steps), obs,
                            ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(N.data_ptr()), optp, stream)


CASES = [
    # M, couplings, dt, steps, prec, options
    (20, workloads.ladder(10), 0.05, 40, spq.SPIN_C64, None),          # tiled, half-tile exchanges
    (17, workloads.star(17, 5), 0.02, 9, spq.SPIN_C64, None),           # smaller: tiled
    (18, workloads.ladder(9), 0.05, 30, spq.SPIN_C128, spq.Options(exchange=1)),
    (16, workloads.ladder(8), 0.05, 12, spq.SPIN_C128, None),
    (12, workloads.ladder(6), 0.05, 20, spq.SPIN_C64, None),            # one workgroup
    (15, workloads.ladder(7) + [(0, 14, 0.0, 0.3)], 0.05, 5, spq.SPIN_C64, spq.Options(schedule=1)),
]


def _set_up(lib, torch):
    """The first call on a device looks up the address of its fixed array
    (HIP places the array on the device then); make that call first."""
    M, J, dt, steps = 10, workloads.ladder(5), 0.05, 2
    psi = torch.empty(2 ** M, dtype=torch.complex64, device="cuda")
    P = torch.zeros(steps + 1, dtype=torch.float64, device="cuda")
    spq.spin_prepare_plan(spq.SPIN_C64, M, J, dt, steps, 0, None)
    spq.spin_init_random_phase(psi, M, 0, 1)
    N = torch.zeros_like(P)
    assert _run(lib, "spin_trotter_evolve_noalloc", psi, spq.SPIN_C64, M, J, dt, steps, 0, P, N, None,
                torch) == 0
    torch.cuda.synchronize()


def test_noalloc_matches_evolve_ex_on_consecutive_calls():
    import torch
    assert torch.cuda.is_available()
    lib = spq.load_library()
    _set_up(lib, torch)
    for M, J, dt, steps, prec, opt in CASES:
        note("noalloc", M, prec, steps)
        dtype = torch_dtype(prec)
        psi = torch.empty(2 ** M, dtype=dtype, device="cuda")
        psi_ref = torch.empty_like(psi)
        P = torch.full((steps + 1,), float("nan"), dtype=torch.float64, device="cuda")
        N = torch.full_like(P, float("nan"))
        Pr, Nr = torch.full_like(P, float("nan")), torch.full_like(P, float("nan"))
        spq.spin_prepare_plan(prec, M, J, dt, steps, 0, opt)
        spq.spin_init_random_phase(psi_ref, M, 0, 11)
        assert _run(lib, "spin_trotter_evolve_ex", psi_ref, prec, M, J, dt, steps, 0, Pr, Nr, opt, torch) == 0
        spq.spin_init_random_phase(psi, M, 0, 11)
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        rc = _run(lib, "spin_trotter_evolve_noalloc", psi, prec, M, J, dt, steps, 0, P, N, opt, torch)
        assert rc == 0, spq.spin_last_error()
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        assert free1 == free0
        assert np.array_equal(P.cpu().numpy(), Pr.cpu().numpy())
        assert np.array_equal(N.cpu().numpy(), Nr.cpu().numpy())
        assert torch.equal(psi, psi_ref)


def test_noalloc_refuses_what_it_cannot_serve_without_allocating():
    import torch
    lib = spq.load_library()
    M, J, dt, steps = 19, workloads.ladder(9) + [(0, 18, 0.0, 0.7)], 0.05, 7
    psi = torch.empty(2 ** M, dtype=torch.complex64, device="cuda")
    P = torch.zeros(steps + 1, dtype=torch.float64, device="cuda")
    N = torch.zeros_like(P)
    spq.spin_init_random_phase(psi, M, 0, 3)
    before = psi.clone()
    # no prepared plan for these arguments
    assert _run(lib, "spin_trotter_evolve_noalloc", psi, spq.SPIN_C64, M, J, dt, steps, 0, P, N, None,
                torch) == spq.SPIN_EUNSUPPORTED
    assert "spin_prepare_plan" in spq.spin_last_error()
    # graph capture
    g = spq.Options(use_graph=1)
    spq.spin_prepare_plan(spq.SPIN_C64, M, J, dt, steps, 0, g)
    assert _run(lib, "spin_trotter_evolve_noalloc", psi, spq.SPIN_C64, M, J, dt, steps, 0, P, N, g,
                torch) == spq.SPIN_EUNSUPPORTED
    torch.cuda.synchronize()
    assert torch.equal(psi, before)
