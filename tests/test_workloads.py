"""Input generators: the paper's printed example systems are read as printed (Sec. 4.1, 4.2)."""
import numpy as np

import workloads


def test_paper_systems_as_printed():
    dimer = workloads.paper_system("abeta_dimer")
    sp = dimer.systems[0]
    assert sp.chain_len == [9, 9] and dimer.box_kind == workloads.BOX_SPHERE
    assert dimer.box_len == 40.0
    letters = "".join("A" if t == workloads.TYPE_A else "B" for t in sp.types)
    assert letters == "BBBBBAAAB" * 2
    for name, first in (("cross_human", "BBBABAAABB"), ("cross_rat", "BBBABAAAAA")):
        wl = workloads.paper_system(name)
        sp = wl.systems[0]
        assert sp.chain_len == [10, 10, 9, 9] and wl.box_len == 20.0
        letters = "".join("A" if t == workloads.TYPE_A else "B" for t in sp.types)
        assert letters == first * 2 + "BBBBBAAAB" * 2
        assert wl.pivot_per_sweep >= 1 and wl.rotate_per_sweep >= 1 and wl.rigid_per_sweep >= 1


def test_paper_systems_start_inside_their_spheres():
    for name in workloads.PAPER_SYSTEMS:
        wl = workloads.paper_system(name)
        pos = workloads.initial_positions(wl)[0]
        assert np.max(np.linalg.norm(pos, axis=1)) < wl.box_len
        bonds = np.linalg.norm(np.diff(pos, axis=0), axis=1)
        ends = np.cumsum(wl.systems[0].chain_len)[:-1] - 1
        assert np.allclose(np.delete(bonds, ends), 1.0)
