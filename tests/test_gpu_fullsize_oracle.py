"""Whole-state parity at the benchmark sizes against the oracle's full loop.

The plain C FP64 loop of the oracle (one pass over the state per factor,
OpenMP over amplitude pairs) runs the first steps of
* the 2 x 15 XY ladder, M = 30 (a 16 GiB complex128 state on the host), and
* the all-to-all star, M = 28 (4 GiB),
from the same random-phase state the GPU writes.  Every P[k] and N[k] of
the observable of Eq. (2) (P = 2(W - 1/2), section "Testing the quantum
parallelism") and every amplitude of the final state are compared with the
HIP path, for each launch shape the benchmark picks between: 1e-10 in FP64,
1e-4 in FP32 (P absolute; amplitudes relative to the largest modulus).

The oracle's state is copied to the device once and the element-by-element
differences are taken there in chunks (test plumbing only; the values come
from the oracle).  The 20-step comparison on the ladder is the run length of
the short benchmark run (a plan of one 20-step block).
"""
import numpy as np
import pytest

import workloads
from oracle import cref
import paper_0710_3747_amd as spq
from gpu_helpers import TOL_P, gpu_evolve, note

pytestmark = pytest.mark.gpu
C64, C128 = spq.SPIN_C64, spq.SPIN_C128
TOL_PSI = {C128: 1e-10, C64: 1e-4}
TOL_N = {C128: 1e-10, C64: 1e-4}


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    spq.load_library()
    cref.build(force=False)
    yield
    torch.cuda.empty_cache()


class OracleRun:
    """The oracle's Strang loop on one workload, advanced on demand: holds P
    and N of steps 0..k and the state after k steps (host, complex128), plus
    a device copy of that state for the comparisons."""

    def __init__(self, M, J, dt, seed):
        self.M, self.J, self.dt, self.seed = M, J, dt, seed
        self.reset()

    def reset(self):
        self.psi = cref.init_random_phase(self.M, 0, self.seed)
        P0, N0 = cref.trotter_run(self.psi, self.M, self.J, self.dt, 0, 0)
        self.P, self.N, self.k = list(P0), list(N0), 0
        self.dev = None

    def at(self, k):
        import torch
        if k < self.k:
            self.reset()
        if k > self.k:
            note("oracle", self.M, "steps", self.k, "->", k)
            P, N = cref.trotter_run(self.psi, self.M, self.J, self.dt, k - self.k, 0)
            self.P += list(P[1:])
            self.N += list(N[1:])
            self.k = k
            self.dev = None
        if self.dev is None:
            self.dev = None
            torch.cuda.empty_cache()
            self.dev = torch.from_numpy(self.psi).cuda()
        return np.array(self.P), np.array(self.N), self.dev

    def release(self):
        self.dev = None
        self.psi = None


def state_error(psi_t, want_t, chunk=1 << 26):
    """max |psi - want| / max |want| over the whole state, in chunks."""
    import torch
    err = scale = 0.0
    for s in range(0, want_t.numel(), chunk):
        w = want_t[s:s + chunk]
        g = psi_t[s:s + chunk].to(torch.complex128)
        err = max(err, float((g - w).abs().max()))
        scale = max(scale, float(w.abs().max()))
    return err / scale


def check_against(orc, prec, steps, opts):
    import torch
    Pw, Nw, want = orc.at(steps)
    note("gpu", orc.M, prec, opts, steps)
    P, N, _, t = gpu_evolve(prec, orc.M, orc.J, orc.dt, steps, 0, seed=orc.seed, opts=opts,
                            keep_state=False)
    dP = np.abs(P - Pw).max()
    dN = np.abs(N - Nw).max()
    dpsi = state_error(t, want)
    del t
    torch.cuda.empty_cache()
    assert dP < TOL_P[prec], f"max |dP| {dP:.3e}"
    assert dN < TOL_N[prec], f"max |dN| {dN:.3e}"
    assert dpsi < TOL_PSI[prec], f"state rel err {dpsi:.3e}"


@pytest.fixture(scope="module")
def ladder30():
    L, dt, _, seed = workloads.LADDER_CONFIGS["ladder_2x15"]
    orc = OracleRun(2 * L, workloads.ladder(L), dt, seed)
    yield orc
    orc.release()


# the default shapes (half-tile exchanges), then shapes the autotuner chooses
# between for the benchmark (tile bits, register bits, coalescing bits, and
# exchange 1 = whole tiles where given)
LADDER_SHAPES = [(C128, None), (C64, None), (C64, (14, 5, 5)), (C64, (14, 5, 6)), (C64, (14, 6, 4)),
                 (C64, (14, 5, 4, 1)), (C64, (14, 4, 4, 1)), (C128, (13, 4, 4, 1)), (C128, (14, 5, 4))]


def _shape_id(p, s):
    name = "c64" if p == C64 else "c128"
    if s is None:
        return name + "-default"
    return name + "-k%d-r%d-c%d" % s[:3] + ("-whole" if len(s) > 3 and s[3] == 1 else "")


LADDER_IDS = [_shape_id(p, s) for p, s in LADDER_SHAPES]


def _opts(shape):
    if shape is None:
        return None
    return dict(zip(("tile_bits", "reg_bits", "coalesce_bits", "exchange"), shape))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,shape", LADDER_SHAPES, ids=LADDER_IDS)
def test_ladder_2x15_three_steps_whole_state(ladder30, prec, shape):
    """2 x 15 ladder (M = 30), 3 steps: every P[k], N[k] and amplitude."""
    check_against(ladder30, prec, 3, _opts(shape))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [C64, C128], ids=["c64", "c128"])
def test_ladder_2x15_twenty_steps_whole_state(ladder30, prec):
    """2 x 15 ladder (M = 30), 20 steps (the short benchmark run's plan), the
    default shapes: every P[k], N[k] and amplitude."""
    check_against(ladder30, prec, 20, None)


@pytest.fixture(scope="module")
def star28():
    cfg = workloads.STAR_M28
    orc = OracleRun(cfg["M"], workloads.star_m28(), cfg["dt"], cfg["seed"])
    yield orc
    orc.release()


STAR_SHAPES = [(C128, None), (C64, None), (C64, (14, 6, 4)), (C128, (14, 5, 4))]
STAR_IDS = [_shape_id(p, s) for p, s in STAR_SHAPES]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,shape", STAR_SHAPES, ids=STAR_IDS)
def test_star_28_two_steps_whole_state(star28, prec, shape):
    """Star M = 28 (378 couplings in the workload's block order), 2 steps:
    every P[k], N[k] and amplitude."""
    check_against(star28, prec, 2, _opts(shape))
