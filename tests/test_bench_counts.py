"""The algorithmic work counts bench.py divides by time: pair and angle-term counts checked by
enumerating the beads of the workloads (CPU only)."""
import itertools

import numpy as np

import bench
import workloads


def _nonbonded_pairs(chain_len):
    chain = np.concatenate([[c] * n for c, n in enumerate(chain_len)])
    n = len(chain)
    return sum(1 for i, j in itertools.combinations(range(n), 2)
               if not (chain[i] == chain[j] and j == i + 1))


def test_differentiation_counts_match_enumeration():
    for lens in (workloads.cross_seeding().systems[0].chain_len, [3], [13], [9, 9, 9, 9]):
        pairs = _nonbonded_pairs(lens)
        angles = sum(max(0, n - 2) for n in lens) + sum(max(0, n - 3) for n in lens)
        fwd, bwd = bench.differentiation_flops_per_config(lens, periodic=True)
        assert fwd == pairs * 23 + angles * 25
        assert bwd == pairs * 37 + angles * 58
    assert _nonbonded_pairs(workloads.cross_seeding().systems[0].chain_len) == 2782


def test_partners_per_move_match_enumeration():
    """A single-bead move of bead b changes its pairs with every bead except itself and its bonded
    neighbours; averaged over the beads of a chain this is the partner count of the formula."""
    for n in (13, 34, 55):
        partners = []
        for b in range(n):
            bonded = (b > 0) + (b < n - 1)
            partners.append(n - 1 - bonded)
        per_pair = 2 * 13 + 2
        expect = np.mean(partners) * per_pair + 50 + 60
        assert abs(bench.algorithmic_flops_per_move(n) - expect) < 1e-9


def test_multichain_move_and_rigid_counts_match_enumeration():
    """Several chains (periodic, torsion): a single-bead move's partners are all beads but itself
    and its bonded neighbours in its own chain; a rigid translation of a chain changes its pairs
    with every bead of the other chains."""
    for wl in (workloads.aggregation(), workloads.cross_seeding()):
        sp = wl.systems[0]
        lens = sp.chain_len
        chain = np.concatenate([[c] * n for c, n in enumerate(lens)])
        n = len(chain)
        partners = []
        for b in range(n):
            bonded = sum(1 for j in (b - 1, b + 1) if 0 <= j < n and chain[j] == chain[b])
            partners.append(n - 1 - bonded)
        torsion = wl.k_tors != 0.0
        expect = np.mean(partners) * (2 * 22 + 2) + 50 + 60 + (56 if torsion else 0)
        assert abs(bench.algorithmic_flops_per_move(n, len(lens), True, torsion) - expect) < 1e-9
        rigid_pairs = np.mean([sum(1 for i in range(n) for j in range(n)
                                   if chain[i] == c and chain[j] != c) for c in range(len(lens))])
        mean_rigid = np.mean([bench.rigid_flops(c, n) for c in lens])
        assert abs(mean_rigid - (rigid_pairs * 46 + 60)) < 1e-9
        assert abs(bench.workload_flops_per_sweep(wl, sp) - (
            n * bench.algorithmic_flops_per_move(n, len(lens), True, torsion)
            + wl.rigid_per_sweep * mean_rigid)) < 1e-6
