"""The host-side split of a mesh into parts (fr_part_host), without a GPU: element counts, ghost
face slots and the exchange lists of every pair of parts, against counts that follow from the
box's geometry and from symmetry (section "Pre-processor Parallelization": faces shared by two
parts are matched by their vertex ids on both sides)."""
import numpy as np
import pytest

from paper_2308_06605_amd import fr
from paper_2308_06605_amd import inputs as I


def _zslab(n, nparts):
    k = np.arange(n ** 3) // (n * n)
    return (k * nparts // n).astype(np.int32)


@pytest.mark.parametrize("n,nparts", [(6, 2), (8, 2), (9, 3)])
def test_slab_split_counts(n, nparts):
    """A periodic n^3 box cut into z-slabs: every part has n^3/nparts elements and shares two
    n x n layers of faces (one with each z-neighbour; both with the same part when there are two)."""
    m = I.box_mesh(n, q=1)
    part = _zslab(n, nparts)
    for q in range(nparts):
        nl, ng, ns, nr = fr.partition_host(m, 3, part, q)
        assert nl == n ** 3 // nparts
        assert ng == 2 * n * n
        assert ns.sum() == nr.sum() == 2 * n * n
        assert ns[q] == nr[q] == 0
        if nparts == 2:
            assert ns[1 - q] == 2 * n * n
        else:
            assert ns[(q + 1) % nparts] == ns[(q - 1) % nparts] == n * n


@pytest.mark.parametrize("seed", [0, 1])
def test_random_split_is_symmetric(seed):
    """Any element -> part map: part a sends to b exactly as many faces as b receives from a,
    and the shared faces equal the element pairs across the cut counted from the mesh itself."""
    n = 5
    m = I.box_mesh(n, q=2, curve_amp=0.05, curve_mode="mixed")
    m, _ = I.scramble_mesh(m, seed=seed)
    rng = np.random.default_rng(seed)
    nparts = 3
    part = rng.integers(0, nparts, size=m.n_elem).astype(np.int32)
    _, _, ftab, _, _ = fr.geometry_host(m, 2)
    cut = np.zeros((nparts, nparts), dtype=np.int64)
    for eL, eR, _, _ in ftab:
        a, b = part[eL], part[eR]
        if a != b:
            cut[a, b] += 1
            cut[b, a] += 1
    ns_all, nr_all = [], []
    for q in range(nparts):
        nl, ng, ns, nr = fr.partition_host(m, 2, part, q)
        assert nl == (part == q).sum()
        assert ng == nr.sum()
        ns_all.append(ns)
        nr_all.append(nr)
    S, Rv = np.array(ns_all), np.array(nr_all)
    assert np.array_equal(S, Rv.T)
    assert np.array_equal(S, cut)


def test_bad_part_maps_are_rejected():
    m = I.box_mesh(4, q=1)
    part = np.zeros(m.n_elem, dtype=np.int32)
    part[0] = 2  # part 1 is empty
    with pytest.raises(fr.FRError):
        fr.partition_host(m, 2, part, 1)
    part[0] = -1
    with pytest.raises(fr.FRError):
        fr.partition_host(m, 2, part, 0)


def test_block_map_of_the_partition_benchmark():
    """partbench's block map: a 2x2x2 cut of a 6^3 box gives eight parts of 27 elements, each a
    3x3x3 box of elements, part index bx-fastest."""
    from paper_2308_06605_amd import partbench as PB

    n = 6
    part = PB.block_map(n, (2, 2, 2))
    assert np.array_equal(np.bincount(part), np.full(8, 27))
    e = np.arange(n ** 3)
    ie, je, ke = e % n, (e // n) % n, e // (n * n)
    assert np.array_equal(part, (ie // 3) + 2 * ((je // 3) + 2 * (ke // 3)))
    assert np.array_equal(np.unique(PB.block_map(n, (3, 1, 2))), np.arange(6))
