"""Pins of the oracle's Monte Carlo: incremental Delta E against full recomputation, bond
preservation, determinism of the counter-based streams, and the flat-weight stationary law
against exact quadrature (N = 3) and iid sampling of bond directions (N = 4)."""
import numpy as np
import pytest

import workloads

CP = workloads.C_LJ_PAPER


def _flat(orc, sp, wl):
    return orc.Weights(sp.e_lo, wl.bin_width, sp.n_bins)


@pytest.mark.parametrize("make", [lambda: workloads.single_chain(),
                                  lambda: workloads.batched_chains(n_seq=2),
                                  lambda: workloads.aggregation(),
                                  lambda: workloads.cross_seeding()])
def test_incremental_delta_e_matches_full_energy(orc, make):
    wl = make()
    sp = wl.systems[-1]
    s = orc.System.from_workload(wl, len(wl.systems) - 1)
    pos0 = workloads.initial_positions(wl)[-1]
    w = orc.Walker(s, pos0, 0, wl.seed)
    H = np.zeros(sp.n_bins, dtype=np.uint64)
    w.run(_flat(orc, sp, wl), orc.move_params(wl), 60, H, check_every=1)
    _, _, scale = s.energy_parts(w.pos)
    assert w.counters.max_drift <= 1e-10 * max(scale, 1.0)
    assert w.counters.accepted > 0.05 * w.counters.moves
    assert w.energy == pytest.approx(s.energy(w.pos), abs=1e-10 * max(scale, 1.0))
    assert int(H.sum()) == w.counters.moves + w.counters.rigid_moves
    if sp.n_chains > 1:
        assert w.counters.rigid_moves == 60 * wl.rigid_per_sweep


def _bond_lengths(pos, chain_len):
    out, off = [], 0
    for n in chain_len:
        out.append(np.linalg.norm(np.diff(pos[off:off + n], axis=0), axis=1))
        off += n
    return np.concatenate(out)


@pytest.mark.parametrize("make", [lambda: workloads.single_chain(),
                                  lambda: workloads.cross_seeding()])
def test_bonds_preserved(orc, make):
    wl = make()
    sp = wl.systems[0]
    s = orc.System.from_workload(wl)
    w = orc.Walker(s, workloads.initial_positions(wl)[0], 3, wl.seed)
    H = np.zeros(sp.n_bins, dtype=np.uint64)
    w.run(_flat(orc, sp, wl), orc.move_params(wl), 2000, H)
    assert np.max(np.abs(_bond_lengths(w.pos, sp.chain_len) - 1.0)) < 1e-12


def test_crankshaft_keeps_next_nearest_distance(orc):
    # a 3-bead chain whose middle bead can only move by crankshaft: |x2 - x0| never changes
    s = orc.System([3], np.array([0, 0, 0], np.uint8), CP)
    pos = np.array([[0.0, 0, 0], [1.0, 0, 0], [1.5, np.sqrt(0.75), 0]])
    d0 = np.linalg.norm(pos[2] - pos[0])
    w = orc.Walker(s, pos, 0, 99)
    W = orc.Weights(-12.0, 0.05, 300)
    H = np.zeros(300, np.uint64)
    mv = dict(crank_max=np.pi / 3, cap_rho=0.0, trans_max=0.0, rigid_per_sweep=0)
    # cap_rho = 0 makes end moves the identity, so only the crankshaft changes coordinates
    w.run(W, mv, 500, H)
    assert np.linalg.norm(w.pos[2] - w.pos[0]) == pytest.approx(d0, abs=1e-13)
    assert not np.allclose(w.pos[1], pos[1])


def test_resume_is_bit_identical(orc):
    wl = workloads.aggregation()
    sp = wl.systems[0]
    s = orc.System.from_workload(wl)
    p0 = workloads.initial_positions(wl)[0]
    W = _flat(orc, sp, wl)
    a = orc.Walker(s, p0, 5, wl.seed)
    Ha = np.zeros(sp.n_bins, np.uint64)
    a.run(W, orc.move_params(wl), 300, Ha)
    b = orc.Walker(s, p0, 5, wl.seed)
    Hb = np.zeros(sp.n_bins, np.uint64)
    b.run(W, orc.move_params(wl), 120, Hb)
    b.run(W, orc.move_params(wl), 180, Hb)
    assert np.array_equal(a.pos, b.pos) and a.energy == b.energy and np.array_equal(Ha, Hb)
    c = orc.Walker(s, p0, 6, wl.seed)           # another walker id: another stream
    Hc = np.zeros(sp.n_bins, np.uint64)
    c.run(W, orc.move_params(wl), 300, Hc)
    assert not np.array_equal(a.pos, c.pos)


def _three_bead_energy_of_cos(orc, s, cvals):
    """E(c) for the 3-bead chain with bond angle cosine c (oracle energy on explicit geometry)."""
    pos = np.zeros((len(cvals), 3, 3))
    pos[:, 1, 0] = 1.0
    pos[:, 2, 0] = 1.0 + cvals
    pos[:, 2, 1] = np.sqrt(np.maximum(0.0, 1.0 - cvals * cvals))
    return s.energy_many(pos)


def _walker_hists(orc, s, sp_len, types, W, mv, n_walkers, n_sweeps, seed, e0pos):
    hs = []
    for i in range(n_walkers):
        w = orc.Walker(s, e0pos, i, seed)
        H = np.zeros(W.n_bins, np.uint64)
        w.run(W, mv, 200, H)                     # burn-in
        H[:] = 0
        w.run(W, mv, n_sweeps, H)
        hs.append(H.astype(np.float64) / H.sum())
    return np.array(hs)


def _coarse(h, edges):
    return np.array([h[..., a:b].sum(axis=-1) for a, b in zip(edges[:-1], edges[1:])]).T


def test_flat_weights_three_beads_match_quadrature(orc):
    """With W = 1 the chain samples iid-uniform bond directions restricted to the window; for
    N = 3 the bond-angle cosine c is uniform on [-1, 1], so bin probabilities follow from E(c)."""
    types = np.array([0, 1, 0], np.uint8)
    s = orc.System([3], types, CP, k_bend=0.25)
    W = orc.Weights(-12.0, 0.05, 300)
    c = -1.0 + (np.arange(4_000_000) + 0.5) * (2.0 / 4_000_000)
    E = _three_bead_energy_of_cos(orc, s, c)
    k = np.floor((E - W.e_lo) / W.bin_width)
    ok = (k >= 0) & (k < W.n_bins)
    p_exact = np.bincount(k[ok].astype(np.int64), minlength=W.n_bins) / ok.sum()
    mv = dict(crank_max=np.pi / 3, cap_rho=0.8, trans_max=0.0, rigid_per_sweep=0)
    start = np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0]])
    hs = _walker_hists(orc, s, [3], types, W, mv, 16, 60000, 77, start)
    # coarse bins of roughly equal exact probability
    cdf = np.cumsum(p_exact)
    edges = np.unique(np.concatenate([[0], np.searchsorted(cdf, np.linspace(0.1, 0.9, 9)) + 1,
                                      [W.n_bins]]))
    pe = _coarse(p_exact, edges)
    ph = _coarse(hs, edges)
    m, se = ph.mean(axis=0), ph.std(axis=0, ddof=1) / np.sqrt(len(ph))
    z = (m - pe) / np.maximum(se, 1e-12)
    assert np.all(np.abs(z) < 5.0), (m, pe, z)


def test_flat_weights_four_beads_match_iid_bonds(orc):
    """N = 4 with bending and torsion: the MCMC histogram at W = 1 against energies of chains
    built from iid uniform bond directions (brute force)."""
    types = np.array([0, 1, 1, 0], np.uint8)
    s = orc.System([4], types, CP, k_bend=0.25, k_tors=0.15)
    W = orc.Weights(-16.0, 0.05, 400)
    rng = np.random.default_rng(2024)
    n = 1_500_000
    v = rng.normal(size=(n, 3, 3))
    v /= np.linalg.norm(v, axis=2, keepdims=True)
    pos = np.zeros((n, 4, 3))
    pos[:, 1:] = np.cumsum(v, axis=1)
    E = s.energy_many(pos)
    k = np.floor((E - W.e_lo) / W.bin_width)
    ok = (k >= 0) & (k < W.n_bins)
    p_iid = np.bincount(k[ok].astype(np.int64), minlength=W.n_bins) / ok.sum()
    mv = dict(crank_max=np.pi / 3, cap_rho=0.8, trans_max=0.0, rigid_per_sweep=0)
    start = np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0]])
    hs = _walker_hists(orc, s, [4], types, W, mv, 16, 40000, 78, start)
    cdf = np.cumsum(p_iid)
    edges = np.unique(np.concatenate([[0], np.searchsorted(cdf, np.linspace(0.1, 0.9, 9)) + 1,
                                      [W.n_bins]]))
    pe = _coarse(p_iid, edges)
    ph = _coarse(hs, edges)
    m, se = ph.mean(axis=0), ph.std(axis=0, ddof=1) / np.sqrt(len(ph))
    se_iid = np.sqrt(pe * (1 - pe) / ok.sum())
    z = (m - pe) / np.sqrt(se ** 2 + se_iid ** 2)
    assert np.all(np.abs(z) < 5.0), (m, pe, z)


def test_planted_sign_error_is_caught(orc):
    """The iid comparison above has teeth: the same MCMC histogram against iid chains whose
    bending enters with the wrong sign fails clearly."""
    types = np.array([0, 1, 1, 0], np.uint8)
    s = orc.System([4], types, CP, k_bend=0.25, k_tors=0.15)
    wrong = orc.System([4], types, CP, k_bend=-0.25, k_tors=0.15)
    W = orc.Weights(-16.0, 0.05, 400)
    rng = np.random.default_rng(2025)
    v = rng.normal(size=(400_000, 3, 3))
    v /= np.linalg.norm(v, axis=2, keepdims=True)
    pos = np.zeros((400_000, 4, 3))
    pos[:, 1:] = np.cumsum(v, axis=1)
    E = wrong.energy_many(pos)
    k = np.floor((E - W.e_lo) / W.bin_width)
    ok = (k >= 0) & (k < W.n_bins)
    p_bad = np.bincount(k[ok].astype(np.int64), minlength=W.n_bins) / ok.sum()
    mv = dict(crank_max=np.pi / 3, cap_rho=0.8, trans_max=0.0, rigid_per_sweep=0)
    hs = _walker_hists(orc, s, [4], types, W, mv, 8, 20000, 79,
                       np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0]]))
    edges = np.arange(0, 401, 20)
    d = np.abs(_coarse(hs, edges).mean(axis=0) - _coarse(p_bad, edges))
    assert d.max() > 0.02
