"""GPU microcanonical analysis (C ABI) against the oracle's numpy implementation, on closed-form
entropies and on weights produced by an oracle MUCA run."""
import math

import numpy as np
import pytest

import workloads
from oracle import analysis as A

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1702_01770_amd as P
    P.load()
    return P


def _same(r_gpu, r_orc, rtol=1e-10, atol=1e-12):
    """Element-wise agreement; points that are NaN on both sides are skipped, but every grid
    must be at least half finite, so that a comparison cannot pass by comparing nothing (F and
    its error are NaN everywhere by definition when no transition temperature exists)."""
    no_bc = isinstance(r_orc["beta_c"], float) and math.isnan(r_orc["beta_c"])
    for k in ("E", "S", "dS", "beta", "dbeta", "cv", "dcv", "F", "dF"):
        a, b = np.asarray(r_gpu[k]), np.asarray(r_orc[k])
        assert a.shape == b.shape, k
        both_nan = np.isnan(a) & np.isnan(b)
        if not (no_bc and k in ("F", "dF")):
            assert np.isfinite(b).sum() >= len(b) / 2, f"{k}: fewer than half the points finite"
        assert np.allclose(a[~both_nan], b[~both_nan], rtol=rtol, atol=atol), k
    for k in ("beta_c", "latent", "barrier", "dbeta_c", "dlatent", "dbarrier"):
        x, y = r_gpu[k], r_orc[k]
        if isinstance(y, float) and math.isnan(y):
            assert math.isnan(x), k
        else:
            assert x == pytest.approx(y, rel=1e-8, abs=1e-12), k


def test_sbend_maxwell(P):
    b0, a, b = 0.8, 0.3, 0.12
    S = lambda e: b0 * e + a * e * e / 2 - b * e ** 4 / 4
    eps, K = 0.004, 2000
    e_lo = -K * eps / 2
    bet, alp = A.coefficients_from_entropy(S, e_lo, eps, K)
    B = np.tile(bet, (4, 1)) + np.random.default_rng(0).normal(scale=1e-4, size=(4, K))
    Al = np.zeros_like(B)
    edges = e_lo + np.arange(K + 1) * eps
    for n in range(4):
        for k in range(K - 2, -1, -1):
            Al[n, k] = Al[n, k + 1] + (B[n, k] - B[n, k + 1]) * edges[k + 1]
    args = (B, Al, e_lo, eps, 0, K, 0, 4, 1, eps)
    kw = dict(beta_c=0.0, tol_beta=1e-3, tol_l=0.0, n_monomers=8)
    rg = P.microcanonical_analyze(*args, **kw)
    ro = A.analyze(*args, **kw)
    _same(rg, ro)
    assert rg["beta_c"] == pytest.approx(b0, abs=1e-3)


def test_given_beta_c_and_intensive(P):
    S = lambda e: -(e - 1.0) ** 2 / 1.2
    bet, alp = A.coefficients_from_entropy(S, -2.0, 0.02, 250)
    B, Al = np.tile(bet, (6, 1)), np.tile(alp, (6, 1))
    args = (B, Al, -2.0, 0.02, 5, 245, 0, 6, 2, 0.02)
    _same(P.microcanonical_analyze(*args, beta_c=1.5, n_monomers=5),
          A.analyze(*args, beta_c=1.5, n_monomers=5))


def test_on_oracle_muca_weights(P, orc):
    wl = workloads.single_chain()
    res = orc.muca(wl, n_iter=12, n_sweeps=3000, walkers=1)
    H = res["hist"][-1]
    vis = np.nonzero(H)[0]
    k_lo, k_hi = int(vis[0]) + 5, int(vis[-1]) - 5
    args = (res["beta"], res["alpha"], wl.systems[0].e_lo, wl.bin_width, k_lo, k_hi, 4, 12, 2,
            2 * wl.bin_width)
    kw = dict(beta_c=0.0, tol_beta=0.05, tol_l=0.0, n_monomers=13)
    _same(P.microcanonical_analyze(*args, **kw), A.analyze(*args, **kw), rtol=1e-9, atol=1e-10)


def test_bad_arguments_rejected(P):
    B = np.zeros((2, 10))
    with pytest.raises(P.MucaError):
        P.microcanonical_analyze(B, B, 0.0, 0.1, 0, 10, 0, 2, 4, 0.1)   # block > iterations
