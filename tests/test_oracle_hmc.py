"""Pins of the hybrid Monte Carlo reference (oracle/hmc.py): exact invariants of the geodesic
leapfrog (unit bonds, time reversibility), its second-order energy error, the generalized
forces against finite differences of U along the sphere and the origin, and the stationary laws
it must reach: iid uniform bonds at flat weights (N = 4) and the canonical law of a 3-bead
chain against quadrature."""
import numpy as np
import pytest

import workloads
from oracle import hmc as HM

CP = workloads.C_LJ_PAPER


def _canonical(orc, T, e_lo=-30.0, K=1200, eps=0.05):
    return orc.Weights(e_lo, eps, K, np.full(K, 1.0 / T), np.zeros(K))


def _chain_walker(orc, wid=3, n_chains=1):
    wl = workloads.aggregation() if n_chains > 1 else workloads.single_chain()
    s = orc.System.from_workload(wl)
    pos = workloads.random_bond_chains(11, 1, wl.systems[0].chain_len, box_len=wl.box_len)[0]
    return s, HM.HmcWalker(s, pos, wid, 1702), wl


@pytest.mark.parametrize("n_chains", [1, 4])
def test_leapfrog_keeps_unit_bonds_and_is_reversible(orc, n_chains):
    s, w, wl = _chain_walker(orc, n_chains=n_chains)
    W = _canonical(orc, 0.7, e_lo=-80.0, K=2400)
    v0 = w.vectors(w.pos)
    m0 = w.momenta(v0, 5)
    v1, m1, pos1 = w.leapfrog(v0, m0, W, 25, 0.02)
    bonds = ~w.first
    assert np.max(np.abs(np.linalg.norm(v1[bonds], axis=1) - 1.0)) < 1e-13
    assert np.max(np.abs(np.sum(v1[bonds] * m1[bonds], axis=1))) < 1e-12
    assert np.max(np.abs(pos1 - w.pos)) > 0.05                   # it did move
    v2, m2, pos2 = w.leapfrog(v1, -m1, W, 25, 0.02)
    assert np.allclose(pos2, w.pos, rtol=0, atol=1e-9)
    assert np.allclose(-m2, m0, rtol=0, atol=1e-9)


def test_energy_error_is_second_order(orc):
    s, w, _ = _chain_walker(orc)
    W = _canonical(orc, 1.0)
    v0 = w.vectors(w.pos)
    m0 = w.momenta(v0, 1)
    H = lambda pos, m: s.energy(pos) + 0.5 * np.sum(m * m)
    H0 = H(w.pos, m0)
    errs = []
    for n, h in ((20, 0.004), (40, 0.002), (80, 0.001)):
        _, m, pos = w.leapfrog(v0, m0, W, n, h)
        errs.append(abs(H(pos, m) - H0))
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_generalized_forces_are_minus_the_gradient_of_u(orc):
    """dU/d(eps) along a tangent turn of bond j (u -> u cos eps + t sin eps) is -G_j . t, and
    along a shift of a chain's first bead it is -G . d (U = E / T)."""
    s, w, _ = _chain_walker(orc, n_chains=4)
    T = 0.8
    W = _canonical(orc, T, e_lo=-80.0, K=2400)
    v = w.vectors(w.pos)
    _, G = w.gen_forces(w.pos, W)
    rng = np.random.default_rng(5)
    U = lambda vv: s.energy(w.positions(vv)) / T
    for j in range(s.n_beads):
        d = rng.normal(size=3)
        vp, vm = v.copy(), v.copy()
        e = 1e-6
        if w.first[j]:
            d /= np.linalg.norm(d)
            vp[j] += e * d
            vm[j] -= e * d
        else:
            t = d - np.dot(d, v[j]) * v[j]
            t /= np.linalg.norm(t)
            vp[j] = v[j] * np.cos(e) + t * np.sin(e)
            vm[j] = v[j] * np.cos(e) - t * np.sin(e)
            d = t
        fd = (U(vp) - U(vm)) / (2 * e)
        assert abs(fd + np.dot(G[j], d)) < 1e-5 * max(1.0, abs(fd)), (j, fd, -np.dot(G[j], d))


def test_flat_weights_give_iid_bonds(orc):
    """U = 0: every trajectory whose end stays in the window is accepted and the bonds perform
    geodesic flow with refreshed momenta, whose stationary law is iid uniform bonds (restricted
    to the window): the energy law of a 4-bead chain with bending and torsion terms against
    chains built from iid unit bonds."""
    types = np.array([0, 1, 1, 0], np.uint8)
    s = orc.System([4], types, CP, k_bend=0.25, k_tors=0.15)
    W = orc.Weights(-16.0, 0.05, 400)
    rng = np.random.default_rng(4242)
    n = 1_000_000
    vv = rng.normal(size=(n, 3, 3))
    vv /= np.linalg.norm(vv, axis=2, keepdims=True)
    pos = np.zeros((n, 4, 3))
    pos[:, 1:] = np.cumsum(vv, axis=1)
    E = s.energy_many(pos)
    k = np.floor((E - W.e_lo) / W.bin_width)
    ok = (k >= 0) & (k < W.n_bins)
    p_iid = np.bincount(k[ok].astype(np.int64), minlength=W.n_bins) / ok.sum()
    start = np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0]])
    hs = []
    for i in range(12):
        w = HM.HmcWalker(s, start, i, 83)
        H = np.zeros(W.n_bins, np.uint64)
        w.run(W, 50, 4, 0.3)
        w.run(W, 1500, 4, 0.3, hist=H)
        assert w.accepted + w.window_rejects == w.traj     # U = 0: only the window rejects
        hs.append(H.astype(np.float64) / H.sum())
    hs = np.array(hs)
    cdf = np.cumsum(p_iid)
    edges = np.unique(np.concatenate([[0], np.searchsorted(cdf, np.linspace(0.1, 0.9, 9)) + 1,
                                      [W.n_bins]]))
    pe = np.array([p_iid[a:b].sum() for a, b in zip(edges[:-1], edges[1:])])
    ph = np.array([hs[:, a:b].sum(axis=1) for a, b in zip(edges[:-1], edges[1:])]).T
    m, se = ph.mean(axis=0), ph.std(axis=0, ddof=1) / np.sqrt(len(ph))
    z = (m - pe) / np.sqrt(se ** 2 + pe * (1 - pe) / ok.sum())
    assert np.all(np.abs(z) < 5.0), (m, pe, z)


def test_canonical_law_of_three_beads(orc):
    """ln W = -E / T: hybrid Monte Carlo alone reproduces the canonical law of a 3-bead chain
    (energy a function of the bond-angle cosine, uniform under the reference measure)."""
    T = 1.0
    types = np.array([0, 1, 0], np.uint8)
    s = orc.System([3], types, CP, k_bend=0.25)
    K = 300
    W = orc.Weights(-12.0, 0.05, K, np.full(K, 1.0 / T), np.zeros(K))
    nq = 2_000_000
    c = -1.0 + (np.arange(nq) + 0.5) * (2.0 / nq)
    pos = np.zeros((nq, 3, 3))
    pos[:, 1, 0] = 1.0
    pos[:, 2, 0] = 1.0 - c
    pos[:, 2, 1] = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    E = s.energy_many(pos)
    k = np.floor((E - W.e_lo) / W.bin_width)
    ok = (k >= 0) & (k < K)
    p_exact = np.bincount(k[ok].astype(np.int64), weights=np.exp(-E[ok] / T), minlength=K)
    p_exact /= p_exact.sum()
    start = np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0]])
    hs = []
    for i in range(12):
        w = HM.HmcWalker(s, start, i, 85)
        H = np.zeros(K, np.uint64)
        w.run(W, 50, 5, 0.15)
        w.run(W, 2000, 5, 0.15, hist=H)
        assert 0.5 < w.accepted / w.traj < 1.0
        hs.append(H.astype(np.float64) / H.sum())
    hs = np.array(hs)
    cdf = np.cumsum(p_exact)
    edges = np.unique(np.concatenate([[0], np.searchsorted(cdf, np.linspace(0.1, 0.9, 9)) + 1,
                                      [K]]))
    pe = np.array([p_exact[a:b].sum() for a, b in zip(edges[:-1], edges[1:])])
    ph = np.array([hs[:, a:b].sum(axis=1) for a, b in zip(edges[:-1], edges[1:])]).T
    m, se = ph.mean(axis=0), ph.std(axis=0, ddof=1) / np.sqrt(len(ph))
    z = (m - pe) / np.maximum(se, 1e-12)
    assert np.all(np.abs(z) < 5.0), (m, pe, z)
