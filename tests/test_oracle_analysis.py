"""Pins of the oracle's microcanonical analysis (Eqs. 4-8, Sec. 3.3) on entropies with closed-form
caloric curves, specific heats and Maxwell constructions."""
import math

import numpy as np
import pytest

from oracle import analysis as A


def _hist(S_func, e_lo, eps, K, n_iter=4, jitter=None):
    b, a = A.coefficients_from_entropy(S_func, e_lo, eps, K)
    B = np.tile(b, (n_iter, 1))
    Al = np.tile(a, (n_iter, 1))
    if jitter is not None:
        Al += jitter[:, None]          # an additive constant per iteration changes nothing
    return B, Al


def test_quadratic_entropy_exact_beta_and_cv():
    mu, sig = 1.0, 0.7
    S = lambda e: -(e - mu) ** 2 / (2 * sig * sig)
    e_lo, eps, K = -2.0, 0.02, 250
    B, Al = _hist(S, e_lo, eps, K, jitter=np.array([0.0, 3.0, -1.5, 7.0]))
    r = A.analyze(B, Al, e_lo, eps, 5, K - 5, 0, 4, 2, eps, beta_c=2.0)
    E = r["E"]
    assert np.allclose(r["beta"], -(E - mu) / sig ** 2, atol=1e-9)
    assert np.allclose(r["cv"], (E - mu) ** 2 / sig ** 2, atol=1e-8)
    assert np.all(r["dbeta"] < 1e-12) and np.all(r["dS"] < 1e-12)   # identical blocks
    # S is normalised to 0 at the top grid point; F = E - S / beta_c (Eq. 7)
    assert r["S"][-1] == pytest.approx(0.0, abs=1e-12)
    assert np.allclose(r["F"], E - r["S"] / 2.0, atol=1e-12)


def test_log_entropy_caloric_curve_and_constant_heat_capacity():
    a, e0 = 2.5, -3.0
    S = lambda e: a * np.log(e - e0)
    e_lo, eps, K = -1.0, 0.005, 800
    B, Al = _hist(S, e_lo, eps, K, n_iter=2)
    r = A.analyze(B, Al, e_lo, eps, 2, K - 2, 0, 2, 1, eps, beta_c=1.0)
    E = r["E"]
    assert np.allclose(r["beta"], a / (E - e0), rtol=2e-5)
    assert np.allclose(r["cv"], a, rtol=2e-3)


def test_intensive_units():
    S = lambda e: -(e - 1.0) ** 2 / 2.0
    B, Al = _hist(S, -2.0, 0.02, 250)
    r1 = A.analyze(B, Al, -2.0, 0.02, 5, 245, 0, 4, 4, 0.02, beta_c=1.0, n_monomers=1)
    r5 = A.analyze(B, Al, -2.0, 0.02, 5, 245, 0, 4, 4, 0.02, beta_c=1.0, n_monomers=5)
    assert np.allclose(r5["E"], r1["E"] / 5) and np.allclose(r5["S"], r1["S"] / 5)
    assert np.allclose(r5["beta"], r1["beta"]) and np.allclose(r5["cv"], r1["cv"] / 5)
    assert np.allclose(r5["F"], r1["F"] / 5)


@pytest.mark.parametrize("N", [1, 8])
def test_maxwell_construction_on_symmetric_backbending(N):
    """beta(E) = b0 + a x - b x^3 (x = E - Ec): the equal-area line is beta_c = b0, the outer
    crossings are x = +-sqrt(a/b) and the free-energy barrier is a^2 / (4 b b0)."""
    b0, a, b, Ec = 0.8, 0.3, 0.12, 0.0
    S = lambda e: b0 * (e - Ec) + a * (e - Ec) ** 2 / 2 - b * (e - Ec) ** 4 / 4
    eps = 0.004
    K = 2000
    e_lo = Ec - K * eps / 2
    B, Al = _hist(S, e_lo, eps, K, n_iter=4)
    r = A.analyze(B, Al, e_lo, eps, 0, K, 0, 4, 1, eps, beta_c=0.0, tol_beta=1e-3,
                  tol_l=0.0, n_monomers=N)
    assert r["beta_c"] == pytest.approx(b0, abs=1e-6)
    assert r["latent"] == pytest.approx(2 * math.sqrt(a / b) / N, rel=1e-4)
    assert r["barrier"] == pytest.approx(a * a / (4 * b * b0) / N, rel=1e-3)
    # negative specific heat inside the backbending (Sec. 4.1)
    inside = np.abs(r["E"] * N - Ec) < 0.5 * math.sqrt(a / (3 * b))
    assert np.all(r["cv"][inside] < 0)


def test_no_backbending_gives_no_transition():
    S = lambda e: 2.0 * np.log(e + 5.0)
    B, Al = _hist(S, -4.0, 0.01, 400)
    r = A.analyze(B, Al, -4.0, 0.01, 2, 398, 0, 4, 2, 0.01, beta_c=0.0, tol_beta=1e-4)
    assert math.isnan(r["beta_c"]) and r["latent"] == 0.0


def test_block_errors_from_scattered_iterations():
    rng = np.random.default_rng(0)
    S = lambda e: -(e - 1.0) ** 2 / 2.0
    b, a = A.coefficients_from_entropy(S, -2.0, 0.05, 100)
    noise = rng.normal(scale=0.01, size=(8, 100))
    B = b + noise
    Al = np.zeros_like(B)
    edges = -2.0 + np.arange(101) * 0.05
    for n in range(8):                               # consistent alpha for each noisy row
        for k in range(98, -1, -1):
            Al[n, k] = Al[n, k + 1] + (B[n, k] - B[n, k + 1]) * edges[k + 1]
    r = A.analyze(B, Al, -2.0, 0.05, 3, 97, 0, 8, 2, 0.05, beta_c=1.0)
    # 4 blocks of 2 iterations: the error is the standard error of the 4 block values
    blocks = []
    for blk in range(4):
        rr = A.analyze(B[2 * blk:2 * blk + 2], Al[2 * blk:2 * blk + 2], -2.0, 0.05, 3, 97, 0, 2,
                       2, 0.05, beta_c=1.0)
        blocks.append(rr["beta"])
    blocks = np.array(blocks)
    assert np.allclose(r["beta"], blocks.mean(axis=0), atol=1e-12)
    assert np.allclose(r["dbeta"], blocks.std(axis=0, ddof=1) / 2.0, atol=1e-12)


def _sbend_blocks(b0s, As, b, e_lo, eps, K):
    """One iteration per block; block i has the caloric curve beta = b0_i + a_i x - b x^3."""
    rows_b, rows_a = [], []
    for b0, a in zip(b0s, As):
        S = lambda e, b0=b0, a=a: b0 * e + a * e * e / 2 - b * e ** 4 / 4
        bb, aa = A.coefficients_from_entropy(S, e_lo, eps, K)
        rows_b.append(bb)
        rows_a.append(aa)
    return np.array(rows_b), np.array(rows_a)


@pytest.mark.parametrize("N", [1, 6])
def test_maxwell_jackknife_errors_have_closed_forms(N):
    """Leave-one-block-out jackknife of the Maxwell construction (Sec. 3.3; binning over
    iterations, Sec. 4.1).  Block i carries the S-bend beta_i(E) = b0_i + a_i x - b x^3, so every
    leave-one-out average is again such an S-bend with the mean parameters of the other blocks,
    whose Maxwell line, latent heat and barrier are known exactly: beta_c = b0, latent heat
    2 sqrt(a/b), barrier a^2 / (4 b b0).  For beta_c the jackknife error then equals the standard
    error of the mean of the b0_i (a property of the jackknife for a linear statistic), which
    pins the (nb - 1)/nb factor and the centring independently of the code's own formula."""
    b0s = np.array([0.80, 0.83, 0.78, 0.81, 0.795, 0.82])
    As = np.array([0.30, 0.33, 0.28, 0.31, 0.295, 0.32])
    b = 0.12
    nb = len(b0s)
    eps, K = 0.004, 2400
    e_lo = -K * eps / 2
    B, Al = _sbend_blocks(b0s, As, b, e_lo, eps, K)
    r = A.analyze(B, Al, e_lo, eps, 0, K, 0, nb, 1, eps, beta_c=0.0, tol_beta=1e-3, tol_l=0.0,
                  n_monomers=N)
    m_b0, m_a = b0s.mean(), As.mean()
    assert r["beta_c"] == pytest.approx(m_b0, abs=1e-6)
    assert r["latent"] == pytest.approx(2 * math.sqrt(m_a / b) / N, rel=1e-4)
    assert r["barrier"] == pytest.approx(m_a ** 2 / (4 * b * m_b0) / N, rel=1e-3)
    # beta_c: jackknife of a mean is the standard error of the mean
    se_b0 = b0s.std(ddof=1) / math.sqrt(nb)
    assert r["dbeta_c"] == pytest.approx(se_b0, rel=1e-3)
    # latent heat and barrier: jackknife over the closed-form leave-one-out values
    loo_b0 = (b0s.sum() - b0s) / (nb - 1)
    loo_a = (As.sum() - As) / (nb - 1)
    lat = 2 * np.sqrt(loo_a / b) / N
    bar = loo_a ** 2 / (4 * b * loo_b0) / N

    def jk(v):
        return math.sqrt((nb - 1) / nb * np.sum((v - v.mean()) ** 2))

    assert r["dlatent"] == pytest.approx(jk(lat), rel=2e-3)
    assert r["dbarrier"] == pytest.approx(jk(bar), rel=2e-2)
    # delta method, to first order in the spread of a: d latent = std(a) / sqrt(nb a b) / N
    assert r["dlatent"] == pytest.approx(As.std(ddof=1) / math.sqrt(nb * m_a * b) / N, rel=0.05)


def test_maxwell_jackknife_vanishes_for_identical_blocks():
    B, Al = _sbend_blocks([0.8] * 4, [0.3] * 4, 0.12, -4.0, 0.004, 2000)
    r = A.analyze(B, Al, -4.0, 0.004, 0, 2000, 0, 4, 1, 0.004, beta_c=0.0, tol_beta=1e-3)
    assert r["dbeta_c"] < 1e-9 and r["dlatent"] < 1e-7 and r["dbarrier"] < 1e-7


@pytest.mark.parametrize("maxwell", [False, True])
def test_free_energy_errors_from_tilted_blocks(maxwell):
    """F(E) = E - S(E)/beta_c (Eq. 7) per block; the error is the standard error over blocks
    (Sec. 4.1).  Blocks whose entropies differ by a tilt c_i (E - E_ref) have, after the
    normalisation S(E_ref) = 0, F errors std(c) |E - E_ref| / (N beta_c sqrt(nb)) in intensive
    units: zero at the reference point and growing linearly away from it."""
    cs = np.array([0.0, 0.02, -0.01, 0.015, -0.025])
    nb, N = len(cs), 4
    eps, K = 0.004, 2000
    e_lo = -K * eps / 2
    b0, a, b = 0.8, 0.3, 0.12
    rows_b, rows_a = [], []
    for c in cs:
        S = lambda e, c=c: (b0 + c) * e + a * e * e / 2 - b * e ** 4 / 4
        bb, aa = A.coefficients_from_entropy(S, e_lo, eps, K)
        rows_b.append(bb)
        rows_a.append(aa)
    B, Al = np.array(rows_b), np.array(rows_a)
    kw = dict(beta_c=0.0, tol_beta=1e-3) if maxwell else dict(beta_c=1.7)
    r = A.analyze(B, Al, e_lo, eps, 0, K, 0, nb, 1, eps, n_monomers=N, **kw)
    bc = r["beta_c"]
    if maxwell:
        assert bc == pytest.approx(b0 + cs.mean(), abs=1e-6)
    else:
        assert bc == 1.7
    e_ref = r["E"][-1] * N
    expect = cs.std(ddof=1) * np.abs(r["E"] * N - e_ref) / (N * bc * math.sqrt(nb))
    assert np.allclose(r["dF"], expect, rtol=1e-9, atol=1e-12)
    # and the mean F is that of the mean entropy
    s_mean = r["S"]
    assert np.allclose(r["F"], r["E"] - s_mean / bc, atol=1e-12)
