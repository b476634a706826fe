"""Pins of the oracle's energy (Eqs. 1-3 plus the torsion-like term) on geometries whose
distances and angles are known exactly, on symmetries, and of its gradient by finite differences."""
import numpy as np
import pytest

import workloads

A, B = workloads.TYPE_A, workloads.TYPE_B
CP = workloads.C_LJ_PAPER


def _sys(orc, chain_len, types, **kw):
    return orc.System(chain_len, np.array(types, dtype=np.uint8), CP, **kw)


def test_eq1_coupling_table_through_two_free_beads(orc):
    # two one-bead "chains" at unit distance: E = kappa_inter (1 - C), C from Eq. (1)
    pos = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    expect = {(A, A): 1.0, (B, B): 0.5, (A, B): -0.5, (B, A): -0.5}
    for (t1, t2), c in expect.items():
        s = _sys(orc, [1, 1], [t1, t2], k_inter=4.0, k_intra=0.0)
        assert s.energy(pos) == pytest.approx(4.0 * (1.0 - c), rel=0, abs=1e-15)


@pytest.mark.parametrize("types,c", [((A, A), 1.0), ((B, B), 0.5), ((A, B), -0.5)])
def test_pair_minimum_location_and_depth(orc, types, c):
    s = _sys(orc, [1, 1], types, k_inter=4.0)
    if c < 0:
        # purely repulsive: energy decreases monotonically with distance
        rs = np.linspace(0.8, 3.0, 200)
        es = [s.energy(np.array([[0.0, 0, 0], [r, 0, 0]])) for r in rs]
        assert np.all(np.diff(es) < 0)
        return
    rmin = (2.0 / c) ** (1.0 / 6.0)
    emin = s.energy(np.array([[0.0, 0, 0], [rmin, 0, 0]]))
    assert emin == pytest.approx(-4.0 * c * c / 4.0, rel=1e-13)
    for dr in (1e-3, -1e-3, 0.05, -0.05):
        assert s.energy(np.array([[0.0, 0, 0], [rmin + dr, 0, 0]])) > emin


def test_straight_three_bead_chain(orc):
    s = _sys(orc, [3], [A, B, A], k_bend=0.25, k_intra=4.0)
    pos = np.array([[0.0, 0, 0], [1.0, 0, 0], [2.0, 0, 0]])
    e, parts, _ = s.energy_parts(pos)
    assert parts[0] == 0.0                         # no bend
    assert parts[2] == pytest.approx(4.0 * (2.0 ** -12 - 1.0 * 2.0 ** -6), rel=1e-14)
    assert e == pytest.approx(parts[2], rel=1e-15)


def test_right_angle_bend(orc):
    s = _sys(orc, [3], [B, A, B], k_bend=0.25)
    pos = np.array([[0.0, 0, 0], [1.0, 0, 0], [1.0, 1.0, 0]])
    e, parts, _ = s.energy_parts(pos)
    assert parts[0] == pytest.approx(0.25, rel=1e-15)
    r = np.sqrt(2.0)
    assert parts[2] == pytest.approx(4.0 * (r ** -12 - 0.5 * r ** -6), rel=1e-14)


def test_bend_uses_normalised_bonds(orc):
    s = _sys(orc, [3], [A, A, A], k_bend=1.0, k_intra=0.0)
    # bonds of lengths 2 and 3 at 60 degrees -> 1 - cos = 1/2 regardless of length
    pos = np.array([[0.0, 0, 0], [2.0, 0, 0], [2.0 + 1.5, 1.5 * np.sqrt(3.0), 0]])
    assert s.energy(pos) == pytest.approx(0.5, rel=1e-14)


def test_torsion_trans_and_cis(orc):
    s = _sys(orc, [4], [A, A, A, A], k_bend=0.0, k_tors=0.7, k_intra=0.0)
    trans = np.array([[0.0, 0, 0], [1, 0, 0], [1, 1, 0], [2, 1, 0]], dtype=float)
    cis = np.array([[0.0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], dtype=float)
    perp = np.array([[0.0, 0, 0], [1, 0, 0], [1, 1, 0], [1, 1, 1]], dtype=float)
    assert s.energy(trans) == pytest.approx(0.0, abs=1e-15)    # bond 1 parallel to bond 3
    assert s.energy(cis) == pytest.approx(1.4, rel=1e-15)      # antiparallel: 2 kappa_T
    assert s.energy(perp) == pytest.approx(0.7, rel=1e-15)     # orthogonal: kappa_T


def test_bonded_pairs_excluded_and_all_others_included(orc):
    # 4-bead chain: LJ over pairs (0,2), (1,3), (0,3) only
    s = _sys(orc, [4], [A, A, A, A], k_bend=0.0, k_intra=4.0)
    pos = np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0]], dtype=float)
    phi = lambda r: 4.0 * (r ** -12 - r ** -6)
    assert s.energy(pos) == pytest.approx(2 * phi(2.0) + phi(3.0), rel=1e-14)


def test_intra_vs_inter_couplings(orc):
    pos = np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 1.3, 0], [1, 1.3, 0], [2, 1.3, 0]])
    base = _sys(orc, [3, 3], [A, B, A, B, A, A], k_intra=4.0, k_inter=4.0, k_bend=0.0)
    _, parts, _ = base.energy_parts(pos)
    no_inter = _sys(orc, [3, 3], [A, B, A, B, A, A], k_intra=4.0, k_inter=0.0, k_bend=0.0)
    e2, parts2, _ = no_inter.energy_parts(pos)
    assert parts2[3] == 0.0 and parts2[2] == parts[2]
    doubled = _sys(orc, [3, 3], [A, B, A, B, A, A], k_intra=4.0, k_inter=8.0, k_bend=0.0)
    _, parts3, _ = doubled.energy_parts(pos)
    assert parts3[3] == pytest.approx(2 * parts[3], rel=1e-15)


def test_rigid_motion_invariance(orc):
    wl = workloads.cross_seeding()
    s = orc.System.from_workload(wl)
    s_free = orc.System(wl.systems[0].chain_len, wl.systems[0].types, CP, k_bend=0.25,
                        k_tors=0.1)
    pos = workloads.random_bond_chains(3, 1, wl.systems[0].chain_len)[0] * 1.0
    e0 = s_free.energy(pos)
    rng = np.random.default_rng(5)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    moved = pos @ q.T + np.array([3.3, -7.1, 0.4])
    assert s_free.energy(moved) == pytest.approx(e0, rel=1e-11)
    # periodic box: translating one chain by a lattice vector changes nothing
    pb = workloads.random_bond_chains(4, 1, wl.systems[0].chain_len, box_len=wl.box_len)[0]
    e1 = s.energy(pb)
    shifted = pb.copy()
    shifted[9:18] += np.array([wl.box_len, -2 * wl.box_len, 0.0])
    assert s.energy(shifted) == pytest.approx(e1, rel=1e-12)


def test_minimum_image(orc):
    L = 20.0
    s = _sys(orc, [1, 1], [A, A], k_inter=4.0, box_kind=2, box_len=L)
    near = s.energy(np.array([[0.5, 3.0, 3.0], [L - 0.5, 3.0, 3.0]]))      # image distance 1
    assert near == pytest.approx(0.0, abs=1e-13)                           # 4 (1 - 1)
    s2 = _sys(orc, [1, 1], [A, A], k_inter=4.0, box_kind=2, box_len=L)
    d = 1.25
    e = s2.energy(np.array([[19.5, 0.2, 7.0], [19.5 + d - L, 0.2 + L, 7.0 - 3 * L]]))
    assert e == pytest.approx(4.0 * (d ** -12 - d ** -6), rel=1e-12)


def test_separated_chains_are_additive(orc):
    wl = workloads.cross_seeding()
    sp = wl.systems[0]
    pos = workloads.random_bond_chains(9, 1, sp.chain_len)[0]
    full = orc.System(sp.chain_len, sp.types, CP, k_bend=0.25, k_tors=0.1)
    far = pos.copy()
    e_sum = 0.0
    off = 0
    for c, n in enumerate(sp.chain_len):
        far[off:off + n] += np.array([1e3 * c, 0, 0])
        single = orc.System([n], sp.types[off:off + n], CP, k_bend=0.25, k_tors=0.1)
        e_sum += single.energy(pos[off:off + n])
        off += n
    assert full.energy(far) == pytest.approx(e_sum, rel=1e-10)


@pytest.mark.parametrize("box", [False, True])
def test_gradient_by_finite_differences(orc, box):
    wl = workloads.cross_seeding()
    sp = wl.systems[0]
    L = wl.box_len if box else 0.0
    s = orc.System(sp.chain_len, sp.types, CP, k_bend=0.23, k_tors=0.11,
                   box_kind=2 if box else 0, box_len=L)
    pos = workloads.random_bond_chains(21, 1, sp.chain_len, box_len=L)[0]
    pos *= 1.05                                   # off the unit-bond manifold on purpose
    e, g, gt = s.energy_grad(pos)
    assert e == pytest.approx(s.energy(pos), rel=1e-15)
    h = 1e-6
    rng = np.random.default_rng(3)
    for _ in range(25):
        i, a = rng.integers(0, len(pos)), rng.integers(0, 3)
        p1, p2 = pos.copy(), pos.copy()
        p1[i, a] += h
        p2[i, a] -= h
        fd = (s.energy(p1) - s.energy(p2)) / (2 * h)
        assert g[i, a] == pytest.approx(fd, rel=1e-6, abs=1e-6 * max(1.0, np.abs(g).max()))
    # theta = (C_AB, C_BB, kappa_bend, kappa_tors): E is linear in each
    base = dict(k_bend=0.23, k_tors=0.11)

    def e_at(cab, cbb, kb, kt):
        cl = np.array([[1.0, cab], [cab, cbb]])
        return orc.System(sp.chain_len, sp.types, cl, k_bend=kb, k_tors=kt,
                          box_kind=2 if box else 0, box_len=L).energy(pos)
    th = np.array([-0.5, 0.5, base["k_bend"], base["k_tors"]])
    for t in range(4):
        d = np.zeros(4)
        d[t] = 1.0
        fd = (e_at(*(th + d)) - e_at(*(th - d))) / 2.0
        assert gt[t] == pytest.approx(fd, rel=1e-7, abs=1e-9)
