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
