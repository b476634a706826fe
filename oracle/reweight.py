"""Canonical reweighting of stored MUCA samples and its force-field gradients, plain numpy FP64
-- TEST INFRASTRUCTURE ONLY.

Samples s were drawn with MUCA weight W(E0_s) (Eq. 8, energy E0_s at the sampling parameters).
For parameters theta and inverse temperature beta = 1/T the canonical average is
    <O>_{beta,theta} = sum_s O_s w_s / sum_s w_s,   ln w_s = -beta E_s(theta) - ln W(E0_s)
(the sampling weight stays fixed at E0_s).  Heat capacity C_V = beta^2 (<E^2> - <E>^2).
Gradients with respect to theta follow from differentiating the ratio of sums:
    d<O>/dtheta = <dO/dtheta> - beta (<O dE/dtheta> - <O><dE/dtheta>)
with O = E (dO/dtheta = dE/dtheta) and O = E^2 (dO/dtheta = 2 E dE/dtheta), and
    dC_V/dtheta = beta^2 (d<E^2>/dtheta - 2 <E> d<E>/dtheta).
Reweighting is not part of the paper; it builds on its MUCA weights (Eq. 8).
"""
from __future__ import annotations

import numpy as np


def canonical(E, lnw0, temps):
    """<E>_T and C_V(T) for every temperature (log-sum-exp in FP64)."""
    E = np.asarray(E, dtype=np.float64)
    lnw0 = np.asarray(lnw0, dtype=np.float64)
    mean_e, cv = [], []
    for T in temps:
        b = 1.0 / T
        lw = -b * E - lnw0
        p = np.exp(lw - lw.max())
        p /= p.sum()
        m1 = np.sum(p * E)
        m2 = np.sum(p * E * E)
        mean_e.append(m1)
        cv.append(b * b * (m2 - m1 * m1))
    return np.array(mean_e), np.array(cv)


def canonical_grad(E, dEdtheta, lnw0, temps):
    """d<E>_T/dtheta and dC_V(T)/dtheta, arrays [n_T, n_theta]."""
    E = np.asarray(E, dtype=np.float64)
    G = np.asarray(dEdtheta, dtype=np.float64)
    lnw0 = np.asarray(lnw0, dtype=np.float64)
    d_mean, d_cv = [], []
    for T in temps:
        b = 1.0 / T
        lw = -b * E - lnw0
        p = np.exp(lw - lw.max())
        p /= p.sum()
        m1 = np.sum(p * E)
        m2 = np.sum(p * E * E)
        g = (p[:, None] * G).sum(axis=0)                 # <dE/dtheta>
        eg = (p[:, None] * E[:, None] * G).sum(axis=0)   # <E dE/dtheta>
        e2g = (p[:, None] * (E * E)[:, None] * G).sum(axis=0)
        dm1 = g - b * (eg - m1 * g)
        dm2 = 2.0 * eg - b * (e2g - m2 * g)
        d_mean.append(dm1)
        d_cv.append(b * b * (dm2 - 2.0 * m1 * dm1))
    return np.array(d_mean), np.array(d_cv)
