"""Pins of the oracle's chain moves (the paper's pivotings and Galilean rotations, Sec. 3.2):
rigid-body invariants of each move isolated (single-bead moves switched off by a zero crankshaft
angle and a zero cap radius), bond preservation, and the stationary laws they must leave
invariant: iid bond directions at flat weights (N = 4, pivots alone) and the canonical law of a
3-bead chain (N = 3, all moves) against quadrature."""
import dataclasses

import numpy as np

import workloads

CP = workloads.C_LJ_PAPER
FROZEN = dict(crank_max=0.0, cap_rho=0.0, trans_max=0.0, rigid_per_sweep=0)   # identity moves


def _chains(pos, chain_len):
    off = np.concatenate([[0], np.cumsum(chain_len)])
    return [pos[a:b] for a, b in zip(off[:-1], off[1:])]


def test_rotations_keep_chain_shapes_and_centres(orc):
    wl = workloads.aggregation()
    sp = wl.systems[0]
    s = orc.System.from_workload(wl)
    pos0 = workloads.initial_positions(wl)[0]
    w = orc.Walker(s, pos0, 5, wl.seed)
    H = np.zeros(sp.n_bins, np.uint64)
    W = orc.Weights(sp.e_lo, wl.bin_width, sp.n_bins)
    w.run(W, dict(FROZEN, rotate_per_sweep=2, rotate_max=np.pi / 3), 400, H)
    assert w.counters.rot_accepted > 100 and w.counters.rot_moves == 800
    assert w.counters.accepted == w.counters.moves          # single-bead moves are identities
    for c0, c1 in zip(_chains(pos0, sp.chain_len), _chains(w.pos, sp.chain_len)):
        assert np.allclose(c0.mean(axis=0), c1.mean(axis=0), atol=1e-12)
        d0 = np.linalg.norm(c0[:, None] - c0[None], axis=2)
        d1 = np.linalg.norm(c1[:, None] - c1[None], axis=2)
        assert np.allclose(d0, d1, atol=1e-11)
    assert np.max(np.abs(w.pos - pos0)) > 0.5                 # the chains did turn
    assert w.energy == s.energy(w.pos) or abs(w.energy - s.energy(w.pos)) < 1e-10


def test_pivots_keep_bonds_and_energy(orc):
    wl = dataclasses.replace(workloads.single_chain(), pivot_per_sweep=3)
    sp = wl.systems[0]
    s = orc.System.from_workload(wl)
    w = orc.Walker(s, workloads.initial_positions(wl)[0], 2, wl.seed)
    H = np.zeros(sp.n_bins, np.uint64)
    w.run(orc.Weights(sp.e_lo, wl.bin_width, sp.n_bins), orc.move_params(wl), 2000, H)
    bl = np.linalg.norm(np.diff(w.pos, axis=0), axis=1)
    assert np.max(np.abs(bl - 1.0)) < 1e-12
    _, _, scale = s.energy_parts(w.pos)
    assert abs(w.energy - s.energy(w.pos)) <= 1e-10 * max(1.0, scale)
    assert w.counters.pivot_moves == 6000 and w.counters.pivot_accepted > 600
    assert int(H.sum()) == w.counters.moves + w.counters.pivot_moves


def test_pivots_alone_sample_iid_bonds_at_flat_weights(orc):
    """With single-bead moves frozen, pivots alone must leave the uniform law of the bond
    directions (restricted to the window) invariant and reach it: the energy histogram of a
    4-bead chain with bending and torsion against chains built from iid unit bonds."""
    types = np.array([0, 1, 1, 0], np.uint8)
    s = orc.System([4], types, CP, k_bend=0.25, k_tors=0.15)
    W = orc.Weights(-16.0, 0.05, 400)
    rng = np.random.default_rng(4242)
    n = 1_500_000
    v = rng.normal(size=(n, 3, 3))
    v /= np.linalg.norm(v, axis=2, keepdims=True)
    pos = np.zeros((n, 4, 3))
    pos[:, 1:] = np.cumsum(v, axis=1)
    E = s.energy_many(pos)
    k = np.floor((E - W.e_lo) / W.bin_width)
    ok = (k >= 0) & (k < W.n_bins)
    p_iid = np.bincount(k[ok].astype(np.int64), minlength=W.n_bins) / ok.sum()
    mv = dict(FROZEN, pivot_per_sweep=4, pivot_max=np.pi / 2)
    start = np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0]])
    hs = []
    for i in range(16):
        w = orc.Walker(s, start, i, 79)
        H = np.zeros(W.n_bins, np.uint64)
        w.run(W, mv, 200, H)
        H[:] = 0
        w.run(W, mv, 30000, H)
        hs.append(H.astype(np.float64) / H.sum())
    hs = np.array(hs)
    cdf = np.cumsum(p_iid)
    edges = np.unique(np.concatenate([[0], np.searchsorted(cdf, np.linspace(0.1, 0.9, 9)) + 1,
                                      [W.n_bins]]))
    pe = np.array([p_iid[a:b].sum() for a, b in zip(edges[:-1], edges[1:])])
    ph = np.array([hs[:, a:b].sum(axis=1) for a, b in zip(edges[:-1], edges[1:])]).T
    m, se = ph.mean(axis=0), ph.std(axis=0, ddof=1) / np.sqrt(len(ph))
    se_iid = np.sqrt(pe * (1 - pe) / ok.sum())
    z = (m - pe) / np.sqrt(se ** 2 + se_iid ** 2)
    assert np.all(np.abs(z) < 5.0), (m, pe, z)


def test_canonical_law_of_three_beads_with_pivots(orc):
    """ln W = -E / T (beta_k = 1/T, alpha_k = 0) turns the MUCA sampler into a canonical one.
    A 3-bead chain's energy depends on the bond-angle cosine c alone, uniform on [-1, 1] under
    the reference measure, so P(bin) is the quadrature of exp(-E(c)/T) over the c of the bin."""
    T = 1.0
    types = np.array([0, 1, 0], np.uint8)
    s = orc.System([3], types, CP, k_bend=0.25)
    K = 300
    W = orc.Weights(-12.0, 0.05, K, np.full(K, 1.0 / T), np.zeros(K))
    nq = 4_000_000
    c = -1.0 + (np.arange(nq) + 0.5) * (2.0 / nq)
    pos = np.zeros((nq, 3, 3))
    pos[:, 1, 0] = 1.0
    pos[:, 2, 0] = 1.0 - c                       # bond 2 at angle arccos(c) to bond 1
    pos[:, 2, 1] = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    E = s.energy_many(pos)
    k = np.floor((E - W.e_lo) / W.bin_width)
    ok = (k >= 0) & (k < K)
    p_exact = np.bincount(k[ok].astype(np.int64), weights=np.exp(-E[ok] / T), minlength=K)
    p_exact /= p_exact.sum()
    mv = dict(crank_max=np.pi / 3, cap_rho=0.8, trans_max=0.0, rigid_per_sweep=0,
              pivot_per_sweep=2, pivot_max=np.pi / 2)
    start = np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0]])
    hs = []
    for i in range(16):
        w = orc.Walker(s, start, i, 81)
        H = np.zeros(K, np.uint64)
        w.run(W, mv, 500, H)
        H[:] = 0
        w.run(W, mv, 40000, H)
        hs.append(H.astype(np.float64) / H.sum())
        assert w.counters.pivot_accepted > 0
    hs = np.array(hs)
    cdf = np.cumsum(p_exact)
    edges = np.unique(np.concatenate([[0], np.searchsorted(cdf, np.linspace(0.1, 0.9, 9)) + 1,
                                      [K]]))
    pe = np.array([p_exact[a:b].sum() for a, b in zip(edges[:-1], edges[1:])])
    ph = np.array([hs[:, a:b].sum(axis=1) for a, b in zip(edges[:-1], edges[1:])]).T
    m, se = ph.mean(axis=0), ph.std(axis=0, ddof=1) / np.sqrt(len(ph))
    z = (m - pe) / np.maximum(se, 1e-12)
    assert np.all(np.abs(z) < 5.0), (m, pe, z)
