"""Pins of the oracle's weight recursion (Sec. 2.2: W^0 = 1, W^{n+1} = W^n / H^n, Berg's
accumulated error-weighted recursion), of the flatness statistics (Sec. 4.1), and of a full MUCA
run on the 3-bead chain whose density of states is known by quadrature."""
import numpy as np
import pytest

import workloads

CP = workloads.C_LJ_PAPER


def _lnw(W, e):
    k = np.clip(np.floor((e - W.e_lo) / W.bin_width).astype(int), 0, W.n_bins - 1)
    return -W.beta[k] * e + W.alpha[k]


def test_first_iteration_is_the_simple_recursion(orc):
    W = orc.Weights(-1.0, 0.5, 5)
    H = np.array([10, 20, 40, 40, 10], np.uint64)
    W.berg_update(H)
    # beta_k = ln(H_{k+1}/H_k)/eps, last bin copies its neighbour
    expect = np.array([np.log(2), np.log(2), 0.0, np.log(0.25), 0.0]) / 0.5
    expect[4] = expect[3]
    assert np.allclose(W.beta, expect, rtol=0, atol=1e-15)
    # ln W^{1}(E) - ln W^{1}(E') = -(ln H(E) - ln H(E')) between bin centres k and k+1 is the
    # simple recursion W^{n+1} = W^n / H^n up to the half-bin placement of the slope
    edges = W.e_lo + np.arange(6) * W.bin_width
    lw = _lnw(W, edges[:-1])
    assert np.allclose(np.diff(lw)[:3], -np.log(H[1:4].astype(float) / H[:3]), atol=1e-14)


def test_lnw_is_continuous_at_every_edge(orc):
    rng = np.random.default_rng(4)
    W = orc.Weights(-3.0, 0.1, 40)
    for _ in range(3):
        W.berg_update(rng.integers(1, 1000, size=40).astype(np.uint64))
    e = W.e_lo + np.arange(1, 40) * W.bin_width
    left = -W.beta[:-1] * e + W.alpha[:-1]
    right = -W.beta[1:] * e + W.alpha[1:]
    assert np.allclose(left, right, rtol=0, atol=1e-12)
    assert W.alpha[-1] == 0.0


def test_flat_histogram_is_a_fixed_point(orc):
    W = orc.Weights(0.0, 0.2, 8, beta=np.linspace(1, 2, 8))
    W.alpha[:] = 0.0
    before = W.beta.copy()
    W.berg_update(np.full(8, 500, np.uint64))
    assert np.array_equal(W.beta[:-1], before[:-1])
    assert W.beta[-1] == W.beta[-2]
    assert np.allclose(W.g[:-1], 250.0)


def test_noiseless_histogram_recovers_entropy_slopes_and_weights_average(orc):
    """H_k = c Omega_k W^n_k with ln Omega known: one step gives beta_k equal to the node slope of
    S = ln Omega; repeating the same histogram gives ghat = 1/2 (equal-weight average)."""
    K, eps, e_lo = 30, 0.1, -2.0
    edges = e_lo + np.arange(K + 1) * eps
    S = lambda e: 3.0 * np.log(e + 2.5) + 0.2 * e * e
    rng = np.random.default_rng(8)
    W = orc.Weights(e_lo, eps, K, beta=rng.normal(size=K))
    W.alpha[:] = 0.0
    for k in range(K - 2, -1, -1):               # consistent alpha for the random start
        W.alpha[k] = W.alpha[k + 1] + (W.beta[k] - W.beta[k + 1]) * edges[k + 1]
    lnH = S(edges[:-1]) + _lnw(W, edges[:-1])
    H = np.round(np.exp(lnH - lnH.max() + np.log(1e15))).astype(np.uint64)
    start = W.beta.copy()
    W.berg_update(H)
    slope = (S(edges[1:-1]) - S(edges[:-2])) / eps
    assert np.allclose(W.beta[:-1], slope, rtol=1e-9, atol=1e-9)
    W2 = orc.Weights(e_lo, eps, K, beta=start)
    W2.alpha[:] = 0.0
    W2.berg_update(H)
    mid = W2.beta.copy()
    W2.berg_update(H)                            # same histogram again: ghat = 1/2
    step = (np.log(H[1:].astype(float)) - np.log(H[:-1].astype(float))) / eps
    assert np.allclose(W2.beta[:-1], mid[:-1] + 0.5 * step, rtol=1e-12, atol=1e-12)


def test_empty_bins_keep_beta_and_extend_downward(orc):
    W = orc.Weights(0.0, 1.0, 8, beta=np.full(8, 0.3))
    H = np.array([0, 0, 0, 100, 50, 0, 25, 25], np.uint64)
    W.berg_update(H)
    b3 = 0.3 + np.log(0.5)
    assert W.beta[3] == pytest.approx(b3, abs=1e-15)
    assert W.beta[4] == 0.3 and W.beta[5] == 0.3      # a neighbour is empty: unchanged
    assert W.beta[6] == pytest.approx(0.3, abs=1e-15)  # equal counts: unchanged
    assert np.all(W.beta[:3] == W.beta[3])             # below the lowest visited bin
    assert W.g[4] == 0 and W.g[3] > 0


def test_flatness_statistics(orc):
    assert orc.flatness(np.full(10, 7, np.uint64))[:2] == (0.0, 0.0)
    cv, pk, lo, hi = orc.flatness(np.array([0, 1, 3, 1, 3, 0], np.uint64))
    assert (lo, hi) == (1, 4)
    assert cv == pytest.approx(0.5) and pk == pytest.approx(0.5)
    cv, pk, lo, hi = orc.flatness(np.array([4, 0, 4], np.uint64))   # interior zero counts
    assert cv == pytest.approx(np.sqrt(32 / 9) / (8 / 3)) and pk == pytest.approx(1.0)


def test_muca_flattens_the_exact_three_bead_distribution(orc):
    """End to end on N = 3: after the iterations, the exact bin weights int_bin Omega(E) W(E) dE
    (quadrature over the bond-angle cosine) are flat over the sampled range."""
    # ends A and B: a repulsive pair, so E(c) is monotonic and Omega(E) smooth over the window
    # (an attractive end pair gives Omega a cliff inside one bin, which the recursion with
    # piecewise-linear ln W resolves only slowly)
    types = np.array([0, 0, 1], np.uint8)
    wl = workloads.Workload(name="n3", systems=[workloads.SystemSpec([3], types, -12.0, 300)],
                            walkers_per_system=4, n_iter=14, n_sweeps=40000, seed=31)
    res = orc.muca(wl)
    W = res["weights"]
    s = orc.System.from_workload(wl)
    c = -1.0 + (np.arange(2_000_000) + 0.5) * 1e-6
    pos = np.zeros((len(c), 3, 3))
    pos[:, 1, 0] = 1.0
    pos[:, 2, 0] = 1.0 + c
    pos[:, 2, 1] = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    E = s.energy_many(pos)
    t = (E - W.e_lo) / W.bin_width
    ok = (t >= 0) & (t < W.n_bins)
    k = np.floor(np.where(ok, t, 0)).astype(np.int64)[ok]
    wts = np.exp(_lnw(W, E[ok]) - _lnw(W, E[ok]).max())
    p = np.bincount(k, weights=wts, minlength=W.n_bins)
    H = res["hist"][-1]
    vis = np.nonzero(H)[0]
    inner = np.arange(vis[0] + 3, vis[-1] - 2)
    q = p[inner] / p[inner].mean()
    assert vis[-1] - vis[0] > 50
    assert np.std(q) < 0.04 and np.max(np.abs(q - 1)) < 0.12, (np.std(q), np.max(np.abs(q - 1)))
    cv, peak, _, _ = res["flat"][-1]
    assert cv < 0.15


def test_bounded_recursion_clamps_to_the_inverse_temperature_range(orc):
    """With bounds [beta_min, beta_max] every updated slope is the unbounded update clipped to the
    range, the slopes below the lowest visited bin copy the clipped one, ln W stays continuous,
    and bounds wide enough to hold every slope change nothing."""
    H = np.array([0, 0, 1, 4, 40, 400, 500, 300, 300, 100], np.uint64)
    free = orc.Weights(-5.0, 0.05, 10)
    free.berg_update(H)
    for lo, hi in ((0.0, 5.0), (-1.0, 40.0), (10.0, 30.0)):
        W = orc.Weights(-5.0, 0.05, 10, beta_min=lo, beta_max=hi)
        W.berg_update(H)
        upd = np.nonzero((H[:-1] > 0) & (H[1:] > 0))[0]
        assert np.allclose(W.beta[upd], np.clip(free.beta[upd], lo, hi), rtol=0, atol=1e-14)
        assert np.all(W.beta[:2] == W.beta[2])
        assert W.beta[-1] == W.beta[-2]
        e = W.e_lo + np.arange(1, 10) * W.bin_width
        assert np.allclose(-W.beta[:-1] * e + W.alpha[:-1], -W.beta[1:] * e + W.alpha[1:],
                           rtol=0, atol=1e-12)
        assert np.array_equal(W.g, free.g)
    wide = orc.Weights(-5.0, 0.05, 10, beta_min=-1e3, beta_max=1e3)
    wide.berg_update(H)
    assert np.array_equal(wide.beta, free.beta) and np.array_equal(wide.alpha, free.alpha)
    # a steep tail (1 -> 4 counts) would give beta = ln 4 / 0.05 = 27.7 below the visited range
    assert free.beta[0] == pytest.approx(np.log(4.0) / 0.05)
