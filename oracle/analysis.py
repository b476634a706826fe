"""Microcanonical analysis (the paper's ANALYST module) in plain numpy FP64 -- TEST INFRASTRUCTURE.

From the per-iteration MUCA coefficients {beta_k, alpha_k}_n (Eq. 8) this computes, on a grid of
bin centres, the entropy S(E) (Eq. 4, k_B = 1), the caloric curve beta(E) = dS/dE (Eq. 5), the
specific heat C_V = -(S')^2 / S'' (Eq. 6) and the free energy F(E) = E - S(E)/beta_c (Eq. 7),
with binning error bars over blocks of consecutive iterations (Sec. 4.1) and, when no beta_c is
given, a Maxwell construction on beta(eps) (Sec. 3.3: Tol_Beta, Tol_L).

Readings (the paper names these steps but does not spell them out):
  * S_n(E) = beta_k E - alpha_k with k the bin of E, i.e. minus the continuous piecewise-linear
    ln W_n(E); every iteration is shifted so that S_n(E_ref) = 0 at the top grid point.
  * Block b averages S_n over its `block` iterations; derivatives are central differences of
    step dE on the block average; observables are averaged over blocks, error = std / sqrt(nb).
  * Intensive units divide E, S, C_V and F by the number of monomers.
  * A backbending is a local minimum of beta followed by a local maximum that is higher by more
    than tol_beta (neighbouring pairs separated by a dip smaller than tol_beta are merged).
    beta_c solves the equal-area condition integral_{e1}^{e3} (beta - beta_c) de = 0 between the
    outer crossings e1 < e3 (bisection, beta piecewise linear between grid points); the latent
    heat is e3 - e1 (kept if >= tol_l) and the barrier max f - f(e1) on [e1, e3].  With several
    backbendings the one with the largest latent heat is reported.  Errors of beta_c, latent
    heat and barrier come from a leave-one-block-out jackknife.
"""
from __future__ import annotations

import math

import numpy as np


def s_of_e(beta_n, alpha_n, e_lo, eps, e):
    """S_n(E) = beta_k E - alpha_k for every iteration row; e may be an array."""
    K = beta_n.shape[-1]
    k = np.clip(np.floor((np.asarray(e) - e_lo) / eps).astype(np.int64), 0, K - 1)
    return beta_n[..., k] * e - alpha_n[..., k]


def _observables(S0, Sm, Sp, dE):
    beta = (Sp - Sm) / (2.0 * dE)
    s2 = (Sp - 2.0 * S0 + Sm) / (dE * dE)
    with np.errstate(divide="ignore", invalid="ignore"):
        cv = -beta * beta / s2
    return beta, cv


def _crossing(x0, y0, x1, y1, level):
    return x0 + (level - y0) * (x1 - x0) / (y1 - y0)


def _bends(beta, tol_beta):
    """Backbendings as (index of local minimum, index of the next local maximum)."""
    n = len(beta)
    mins = [i for i in range(1, n - 1) if beta[i] <= beta[i - 1] and beta[i] <= beta[i + 1]]
    maxs = [i for i in range(1, n - 1) if beta[i] >= beta[i - 1] and beta[i] >= beta[i + 1]]
    pairs = []
    for i in mins:
        later = [j for j in maxs if j > i]
        if later and beta[later[0]] - beta[i] > tol_beta:
            pairs.append([i, later[0]])
    merged = []
    for i, j in pairs:
        if merged and i < merged[-1][1]:
            continue                       # starts inside the previous backbending
        if merged and beta[merged[-1][1]] - beta[i] < tol_beta:
            merged[-1][1] = j              # shallow dip: the same backbending continues
        else:
            merged.append([i, j])
    return merged


def _equal_area(eg, beta, i_min, i_max, level):
    """Outer crossings e1 < e3 of beta = level around a backbending and the signed area
    integral_{e1}^{e3} (beta - level) de, beta linear between grid points.  Returns 'high' if
    the level lies above the branch left of the minimum, 'low' if below the branch right of
    the maximum."""
    n = len(beta)
    g = i_min
    while g > 0 and beta[g] < level:
        g -= 1
    if beta[g] < level:
        return "high"
    h = i_max
    while h < n - 1 and beta[h] > level:
        h += 1
    if beta[h] > level:
        return "low"
    e1 = _crossing(eg[g], beta[g], eg[g + 1], beta[g + 1], level) if g < i_min else eg[g]
    e3 = _crossing(eg[h - 1], beta[h - 1], eg[h], beta[h], level) if h > i_max else eg[h]
    xs = [e1] + list(eg[g + 1:h]) + [e3]
    ys = [level] + list(beta[g + 1:h]) + [level]
    area = 0.0
    for a in range(len(xs) - 1):
        area += 0.5 * ((ys[a] - level) + (ys[a + 1] - level)) * (xs[a + 1] - xs[a])
    return e1, e3, area


def maxwell(eg, beta, s, tol_beta, tol_l):
    """Maxwell construction on an intensive caloric curve; returns (beta_c, latent, barrier) of
    the backbending with the largest latent heat, or (nan, 0, 0) if there is none."""
    best = (math.nan, 0.0, 0.0)
    for i_min, i_max in _bends(beta, tol_beta):
        lo, hi = float(beta[i_min]), float(beta[i_max])
        r = None
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            r = _equal_area(eg, beta, i_min, i_max, mid)
            if r == "high":
                hi = mid
            elif r == "low":
                lo = mid
            elif r[2] > 0:
                lo = mid
            else:
                hi = mid
            if hi - lo <= 1e-15 * max(1.0, abs(mid)):
                break
        bc = 0.5 * (lo + hi)
        r = _equal_area(eg, beta, i_min, i_max, bc)
        if isinstance(r, str):
            continue
        e1, e3, _ = r
        latent = e3 - e1
        if latent < tol_l:
            continue
        f = eg - s / bc
        f1 = np.interp(e1, eg, f)
        inside = (eg >= e1) & (eg <= e3)
        barrier = float(np.max(f[inside]) - f1) if inside.any() else 0.0
        if latent > best[1]:
            best = (bc, latent, barrier)
    return best


def analyze(beta_hist, alpha_hist, e_lo, eps, k_lo, k_hi, n_s, n_e, block, dE,
            beta_c=0.0, tol_beta=0.0, tol_l=0.0, n_monomers=1):
    """Microcanonical analysis of iterations [n_s, n_e) on the bin centres of bins [k_lo, k_hi).

    Returns a dict with grid arrays E, S, dS, beta, dbeta, cv, dcv, F, dF (intensive when
    n_monomers > 1) and scalars beta_c, dbeta_c, latent, dlatent, barrier, dbarrier.
    """
    beta_hist = np.asarray(beta_hist, dtype=np.float64)
    alpha_hist = np.asarray(alpha_hist, dtype=np.float64)
    nb = (n_e - n_s) // block
    if nb < 1:
        raise ValueError("need at least one block")
    E = e_lo + (np.arange(k_lo, k_hi) + 0.5) * eps
    e_ref = E[-1]
    Sblk = np.empty((nb, 3, len(E)))
    for b in range(nb):
        rows = slice(n_s + b * block, n_s + (b + 1) * block)
        bn, an = beta_hist[rows], alpha_hist[rows]
        ref = s_of_e(bn, an, e_lo, eps, np.array([e_ref]))[:, 0:1]
        for j, shift in enumerate((0.0, -dE, +dE)):
            Sblk[b, j] = np.mean(s_of_e(bn, an, e_lo, eps, E + shift) - ref, axis=0)
    N = float(n_monomers)

    def curves(S3):
        beta, cv = _observables(S3[0], S3[1], S3[2], dE)
        return S3[0] / N, beta, cv / N

    per_block = [curves(Sblk[b]) for b in range(nb)]
    s_b = np.array([p[0] for p in per_block])
    beta_b = np.array([p[1] for p in per_block])
    cv_b = np.array([p[2] for p in per_block])

    def mean_err(a):
        m = a.mean(axis=0)
        e = a.std(axis=0, ddof=1) / math.sqrt(nb) if nb > 1 else np.zeros_like(m)
        return m, e

    s_m, s_e = mean_err(s_b)
    beta_m, beta_e = mean_err(beta_b)
    cv_m, cv_e = mean_err(cv_b)
    eg = E / N

    S_all = Sblk.mean(axis=0)
    s_all, beta_all, _ = curves(S_all)
    if beta_c > 0:
        bc, latent, barrier = float(beta_c), 0.0, 0.0
        dbc = dlat = dbar = 0.0
    else:
        bc, latent, barrier = maxwell(eg, beta_all, s_all, tol_beta, tol_l)
        jk = []
        if nb > 1:
            for b in range(nb):
                keep = [i for i in range(nb) if i != b]
                s_j, beta_j, _ = curves(Sblk[keep].mean(axis=0))
                jk.append(maxwell(eg, beta_j, s_j, tol_beta, tol_l))
        if jk and not math.isnan(bc):
            jk = np.array(jk)
            fac = (nb - 1) / nb
            dbc, dlat, dbar = (math.sqrt(fac * np.sum((jk[:, i] - jk[:, i].mean()) ** 2))
                               for i in range(3))
        else:
            dbc = dlat = dbar = 0.0
    if math.isnan(bc):
        F_m = np.full_like(eg, np.nan)
        F_e = np.full_like(eg, np.nan)
    else:
        F_m, F_e = mean_err(np.array([eg - s_b[b] / bc for b in range(nb)]))
    return dict(E=eg, S=s_m, dS=s_e, beta=beta_m, dbeta=beta_e, cv=cv_m, dcv=cv_e, F=F_m, dF=F_e,
                beta_c=bc, dbeta_c=dbc, latent=latent, dlatent=dlat, barrier=barrier,
                dbarrier=dbar, n_blocks=nb)


def coefficients_from_entropy(S_func, e_lo, eps, K):
    """MUCA coefficients whose S_n(E) interpolates S(E) linearly between bin edges:
    beta_k = [S(E_{k+1}) - S(E_k)] / eps, alpha_k = beta_k E_k - S(E_k).  Used by the tests to
    feed closed-form entropies into the analysis."""
    edges = e_lo + np.arange(K + 1) * eps
    Sv = S_func(edges)
    beta = (Sv[1:] - Sv[:-1]) / eps
    alpha = beta * edges[:-1] - Sv[:-1]
    return beta, alpha
