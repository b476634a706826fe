"""Two-sample criterion for statistical parity of MUCA estimates (test infrastructure).

Replicas of a curve (S(E), beta(E) or C_V(E) on a grid) from two independent sets of runs, the
GPU's and the oracle's, are compared by a permutation test that is exactly calibrated under the
null hypothesis that every replica of both sets is an independent draw from one distribution
(the replicas are then exchangeable):

  * per grid point, the Mann-Whitney statistic of the two sets (the rank sum of the first set,
    standardised by its null mean and variance), so heavy-tailed or skewed replica
    distributions (trapped MUCA walkers give both) need no normal approximation;
  * three summaries over the grid: max |z| (a local difference), mean z^2 (a broad one) and
    |mean z| (a coherent offset of the whole curve, which max |z| alone cannot see when the grid
    points are strongly correlated);
  * the null distribution of each summary from random relabellings of the pooled replicas (the
    same relabelling for every grid point, so the correlation between points is kept), p-value
    (1 + #{T_perm >= T_obs}) / (1 + n_perm), which is a valid p-value for any n_perm.

Grid points at which some replica is not finite (C_V = -beta^2 / S'' where S'' = 0) are dropped;
the mask depends only on the pooled data, not on the labels, so the test stays exact.  A family
of such tests is run at a Bonferroni-corrected level, so its false-alarm rate is at most the
family level whatever the dependence between curves and summaries.
"""
from __future__ import annotations

import numpy as np

SUMMARIES = ("max_abs_z", "mean_z2", "abs_mean_z")


def _ranks(X):
    """Column-wise ranks 1..n with ties averaged."""
    n, g = X.shape
    order = np.argsort(X, axis=0, kind="stable")
    R = np.empty_like(X, dtype=np.float64)
    cols = np.arange(g)
    R[order, cols] = np.arange(1, n + 1, dtype=np.float64)[:, None]
    # average ties
    Xs = np.take_along_axis(X, order, axis=0)
    for j in np.nonzero((np.diff(Xs, axis=0) == 0).any(axis=0))[0]:
        col = X[:, j]
        vals, inv = np.unique(col, return_inverse=True)
        sums = np.bincount(inv, weights=R[:, j])
        cnts = np.bincount(inv)
        R[:, j] = (sums / cnts)[inv]
    return R


def _summaries(z):
    return np.stack([np.abs(z).max(axis=-1), (z * z).mean(axis=-1), np.abs(z.mean(axis=-1))],
                    axis=-1)


def permutation_test(A, B, n_perm: int = 9999, seed: int = 0) -> dict:
    """p-values of the three summaries for replica arrays A [nA, G] and B [nB, G]."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    X = np.vstack([A, B])
    keep = np.isfinite(X).all(axis=0)
    X = X[:, keep]
    nA, nB = len(A), len(B)
    n = nA + nB
    R = _ranks(X)
    mu = nA * (n + 1) / 2.0
    sd = np.sqrt(nA * nB * (n + 1) / 12.0)

    def z_of(mask_rows):
        return (mask_rows @ R - mu) / sd

    obs_mask = np.zeros(n)
    obs_mask[:nA] = 1.0
    t_obs = _summaries(z_of(obs_mask))
    rng = np.random.default_rng(seed)
    counts = np.zeros(3)
    done = 0
    while done < n_perm:
        m = min(2000, n_perm - done)
        P = np.zeros((m, n))
        idx = np.argsort(rng.random((m, n)), axis=1)[:, :nA]
        np.put_along_axis(P, idx, 1.0, axis=1)
        t = _summaries(z_of(P))
        counts += (t >= t_obs[None, :] - 1e-12).sum(axis=0)
        done += m
    p = (1.0 + counts) / (1.0 + n_perm)
    return dict(zip(SUMMARIES, p)) | dict(stats=dict(zip(SUMMARIES, t_obs)),
                                          n_points=int(keep.sum()))


def family_passes(results: dict, family_alpha: float) -> bool:
    """results: name -> permutation_test output.  Bonferroni over every summary of every curve."""
    n = len(results) * len(SUMMARIES)
    return all(r[s] > family_alpha / n for r in results.values() for s in SUMMARIES)


def compare_curves(gpu: dict, orc: dict, family_alpha: float = 0.01, n_perm: int = 9999,
                   seed: int = 0):
    """gpu, orc: curve name -> replica array.  Returns (passes, results)."""
    res = {k: permutation_test(gpu[k], orc[k], n_perm=n_perm, seed=seed + i)
           for i, k in enumerate(sorted(gpu))}
    return family_passes(res, family_alpha), res
