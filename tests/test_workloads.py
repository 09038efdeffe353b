"""Host checks of the input generators (no GPU, no method arithmetic)."""
import workloads


def test_block_order_is_a_permutation_in_blocks_of_two_groups():
    """The block order lists every coupling once, block after block: each
    coupling sits in the first block (pair of the four site groups) that
    holds both its sites, the blocks appear in order, all six pairs of
    groups are used, and consecutive blocks share a group."""
    M = 28
    J = workloads.star(M, 33)
    B = workloads.block_order(M, J)
    assert sorted(B) == sorted(J) and len(B) == len(J) == M * (M - 1) // 2
    group = [s * 4 // M for s in range(M)]
    path = [tuple(sorted(p)) for p in workloads._K4_PATH]
    assert sorted(path) == [(a, b) for a in range(4) for b in range(a + 1, 4)]
    for p, q in zip(path, path[1:]):
        assert set(p) & set(q)
    idx = [next(n for n, p in enumerate(path) if {group[i], group[j]} <= set(p)) for i, j, a, b in B]
    assert idx == sorted(idx) and set(idx) == set(range(6))
    # within a block the generator's relative order is kept
    for n in range(6):
        blk = [c for c, k in zip(B, idx) if k == n]
        assert blk == [c for c in J if c in blk]


def test_star_m28_is_the_block_ordered_star():
    c = workloads.STAR_M28
    assert workloads.star_m28() == workloads.block_order(c["M"], workloads.star(c["M"], c["coupling_seed"]))
