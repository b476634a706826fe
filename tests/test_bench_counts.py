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
