"""Pins of the oracle's canonical reweighting and its parameter gradients: closed forms for a
two-level system, multiplicity weights, finite differences, and the 3-bead chain whose canonical
averages follow from a 1-D quadrature over the bond-angle cosine."""
import numpy as np
import pytest

import workloads
from oracle import reweight as R

CP = workloads.C_LJ_PAPER
TEMPS = np.linspace(0.1, 1.0, 64)


def test_two_level_closed_form():
    E = np.array([0.0] * 5 + [1.0] * 5)
    m, cv = R.canonical(E, np.zeros(10), TEMPS)
    b = 1.0 / TEMPS
    p = np.exp(-b) / (1.0 + np.exp(-b))
    assert np.allclose(m, p, rtol=1e-13)
    assert np.allclose(cv, b * b * p * (1 - p), rtol=1e-12)


def test_sampling_weights_are_divided_out():
    # level e_i drawn n_i times with ln W0 = ln n_i: every level counts once
    levels = np.array([-2.0, -1.0, 0.5, 3.0])
    counts = np.array([1, 7, 3, 20])
    E = np.repeat(levels, counts)
    lnw0 = np.log(np.repeat(counts, counts).astype(float))
    m, cv = R.canonical(E, lnw0, TEMPS)
    for T, mm, cc in zip(TEMPS, m, cv):
        w = np.exp(-levels / T)
        w /= w.sum()
        e1 = (w * levels).sum()
        assert mm == pytest.approx(e1, rel=1e-12, abs=1e-12)
        assert cc == pytest.approx(((w * levels ** 2).sum() - e1 ** 2) / T ** 2, rel=1e-10)


def test_gradients_by_finite_differences():
    rng = np.random.default_rng(1)
    E = rng.normal(size=500)
    G = rng.normal(size=(500, 4))
    lnw0 = rng.normal(size=500) * 0.5
    dm, dcv = R.canonical_grad(E, G, lnw0, TEMPS)
    h = 1e-6
    for t in range(4):
        mp, cvp = R.canonical(E + h * G[:, t], lnw0, TEMPS)
        mm, cvm = R.canonical(E - h * G[:, t], lnw0, TEMPS)
        assert np.allclose(dm[:, t], (mp - mm) / (2 * h), rtol=1e-5, atol=1e-7)
        assert np.allclose(dcv[:, t], (cvp - cvm) / (2 * h), rtol=1e-5, atol=1e-6)


def _three_bead_quadrature(orc, types, k_bend, temps):
    s = orc.System([3], types, CP, k_bend=k_bend)
    c = -1.0 + (np.arange(400_000) + 0.5) * 5e-6
    pos = np.zeros((len(c), 3, 3))
    pos[:, 1, 0] = 1.0
    pos[:, 2, 0] = 1.0 + c
    pos[:, 2, 1] = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    E = s.energy_many(pos)
    out = []
    for T in temps:
        w = np.exp(-(E - E.min()) / T)
        w /= w.sum()
        m = (w * E).sum()
        out.append((m, ((w * E * E).sum() - m * m) / T ** 2))
    return np.array(out)


def test_reweighted_muca_samples_match_three_bead_quadrature(orc):
    """P9/P10: samples of a MUCA run on N = 3, reweighted to T, against quadrature; the
    kappa_bend gradient against a quadrature finite difference."""
    types = np.array([0, 0, 1], np.uint8)
    wl = workloads.Workload(name="n3", systems=[workloads.SystemSpec([3], types, -12.0, 300)],
                            walkers_per_system=4, n_iter=12, n_sweeps=30000, seed=41)
    res = orc.muca(wl)
    W = res["weights"]
    s = orc.System.from_workload(wl)
    mv = orc.move_params(wl)
    w = res["walkers"][0]
    xs, es = [], []
    H = np.zeros(W.n_bins, np.uint64)
    for _ in range(40000):
        w.run(W, mv, 5, H)
        xs.append(w.pos.copy())
        es.append(w.energy)
    xs, es = np.array(xs), np.array(es)
    k = np.floor((es - W.e_lo) / W.bin_width).astype(int)
    lnw0 = -W.beta[k] * es + W.alpha[k]
    temps = np.array([0.3, 0.5, 1.0])
    m, cv = R.canonical(es, lnw0, temps)
    q = _three_bead_quadrature(orc, types, 0.25, temps)
    assert np.allclose(m, q[:, 0], rtol=0.03, atol=0.01), (m, q[:, 0])
    assert np.allclose(cv, q[:, 1], rtol=0.15, atol=0.02), (cv, q[:, 1])
    G = np.array([s.energy_grad(x)[2] for x in xs])
    dm, _ = R.canonical_grad(es, G, lnw0, temps)
    h = 0.01
    qp = _three_bead_quadrature(orc, types, 0.25 + h, temps)
    qm = _three_bead_quadrature(orc, types, 0.25 - h, temps)
    d_exact = (qp[:, 0] - qm[:, 0]) / (2 * h)
    assert np.allclose(dm[:, 2], d_exact, rtol=0.1, atol=0.05), (dm[:, 2], d_exact)
