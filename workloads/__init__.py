"""Seeded synthetic inputs for the random-phase spin-dynamics path.

This module only *generates inputs* (coupling lists, seeds, problem sizes).
It holds none of the method's arithmetic: no propagator, no phase function,
no observable.  Both the CPU oracle (through the tests) and the HIP library
consume what it returns, so neither side imports the other.

Coupling lists are lists of ``(i, j, a, b)`` tuples with 0-based sites.  The
two-spin term they encode is the one of the paper's section "Spin systems
with different coupling networks":  a_ij I^z_i I^z_j + (b_ij/2)(I^+_i I^-_j +
I^-_i I^+_j).  ``a = 0`` is the XY family used by every configuration here.

Workload families (section "Spin systems with different coupling networks",
items a) and b), and Fig. 2):

* ``ladder(L, bx, by)``: two legs of L sites each.  Leg A is sites 0..L-1,
  leg B is sites L..2L-1; leg bonds (i, i+1) inside each leg (open ends,
  no bond between the two legs' ends), rungs (i, i+L).  Site 0 is an end
  of leg A ("the extreme of a spin ladder", caption of Fig. 3).  List
  order: even leg bonds of both legs, odd leg bonds, then rungs -- three
  layers of mutually commuting factors.
* ``star(M, seed, var_center, var_other)``: every pair coupled; the bonds of
  site 0 are drawn from N(0, var_center), all other bonds from
  N(0, var_other).  The paper's star uses a single Gaussian of variance
  sigma^2; the second variance lets the central spin's bonds be stronger.
  Lexicographic (i, j) order.
* ``star_batch(...)``: many independent stars of uneven size.
* ``block_order(M, couplings)``: the same couplings listed block by block
  (four site groups, every pair of groups once); the M = 28 star is listed
  this way.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "ladder", "chain", "star", "star_batch", "single_bond", "block_order", "star_m28",
    "LADDER_CONFIGS", "STAR_M28", "BATCH_STARS",
]


def ladder(L: int, bx: float = 1.0, by: float = 1.0, a_over_b: float = 0.0):
    """Coupling list of a 2 x L spin ladder (sites 0..2L-1)."""
    if L < 1:
        raise ValueError("ladder needs L >= 1")
    even, odd, rungs = [], [], []
    for leg in (0, 1):
        for i in range(L - 1):
            s = leg * L + i
            (even if i % 2 == 0 else odd).append((s, s + 1, a_over_b * bx, bx))
    for i in range(L):
        rungs.append((i, i + L, a_over_b * by, by))
    return even + odd + rungs


def chain(M: int, b: float = 1.0, a_over_b: float = 0.0):
    """Open chain 0-1-...-(M-1); even bonds first, then odd bonds."""
    even = [(i, i + 1, a_over_b * b, b) for i in range(0, M - 1, 2)]
    odd = [(i, i + 1, a_over_b * b, b) for i in range(1, M - 1, 2)]
    return even + odd


def star(M: int, seed: int, var_center: float = 1.0, var_other: float = 0.1,
         a_over_b: float = 0.0):
    """All-to-all random couplings on M sites (Gaussian, zero mean)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(M):
        for j in range(i + 1, M):
            var = var_center if i == 0 else var_other
            b = float(rng.standard_normal() * np.sqrt(var))
            out.append((i, j, a_over_b * b, b))
    return out


# Blocks of a four-group covering: every pair of groups once, in an order
# where consecutive blocks share a group (a path through the edges of K4).
_K4_PATH = ((0, 1), (1, 3), (0, 3), (0, 2), (2, 3), (1, 2))


def block_order(M: int, couplings):
    """The same couplings listed block by block (a covering order).

    The sites are split into four consecutive groups of nearly equal size;
    block (a, b) holds every listed pair whose sites both lie in groups a
    and b and that no earlier block holds, in the given relative order.
    Blocks follow a path through the six group pairs on which consecutive
    blocks share a group.  With the symmetric step (list order, then
    reversed) a block's factors can be applied together on the union of its
    two groups, so a Trotter step needs about ten such unions instead of one
    per overlapping run of the lexicographic order.  The list order is part
    of the workload: it fixes the Trotter product that every consumer
    evaluates.
    """
    bounds = [round(M * q / 4) for q in range(5)]
    group = [0] * M
    for g in range(4):
        for site in range(bounds[g], bounds[g + 1]):
            group[site] = g
    out, taken = [], set()
    for a, b in _K4_PATH:
        for n, c in enumerate(couplings):
            if n in taken:
                continue
            if {group[c[0]], group[c[1]]} <= {a, b}:
                out.append(c)
                taken.add(n)
    assert len(out) == len(couplings)
    return out


def single_bond(i: int, j: int, b: float = 1.0, a: float = 0.0):
    return [(i, j, a, b)]


def star_batch(n: int, m_lo: int, m_hi: int, size_seed: int,
               coupling_seed0: int, state_seed0: int):
    """``n`` star problems with M drawn uniformly from {m_lo..m_hi}.

    Returns a list of dicts ``{"M", "couplings", "seed"}``; problem r uses
    coupling seed ``coupling_seed0 + r`` and state seed ``state_seed0 + r``.
    """
    rng = np.random.Generator(np.random.PCG64(size_seed))
    Ms = rng.integers(m_lo, m_hi + 1, size=n)
    return [
        {"M": int(M), "couplings": star(int(M), coupling_seed0 + r),
         "seed": state_seed0 + r}
        for r, M in enumerate(Ms)
    ]


# Named workloads: the five problem configurations the path is sized for.
LADDER_CONFIGS = {
    # name: (L, dt, n_steps, state seed)
    "ladder_2x5": (5, 0.05, 400, 1),
    "ladder_2x12": (12, 0.05, 2000, 2),
    "ladder_2x15": (15, 0.05, 1000, 5),
}
# the M = 28 star's couplings (values drawn in lexicographic pair order) are
# listed in the block order of block_order
STAR_M28 = {"M": 28, "coupling_seed": 33, "seed": 3, "dt": 0.02, "n_steps": 1000, "order": "blocks"}


def star_m28():
    """The M = 28 star workload's coupling list (see STAR_M28)."""
    c = STAR_M28
    J = star(c["M"], c["coupling_seed"])
    return block_order(c["M"], J) if c["order"] == "blocks" else J
BATCH_STARS = {"n": 256, "m_lo": 14, "m_hi": 20, "size_seed": 4,
               "coupling_seed0": 2000, "state_seed0": 1000,
               "dt": 0.02, "n_steps": 500}
