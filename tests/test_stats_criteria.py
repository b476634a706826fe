"""The statistical-parity criterion (tests/stats_criteria.py) on the CPU: its p-values are
calibrated (false alarms at the nominal rate on heavy-tailed, strongly correlated synthetic
curves and over random splits of the oracle's own replicas), two disjoint halves of the oracle's
replicas pass it, and it rejects replicas from an oracle with a planted error (a wrong bending
coupling) at the statistics of the stored reference."""
import json
import os
from multiprocessing import Pool

import numpy as np
import pytest

import stats_criteria as sc

HERE = os.path.dirname(os.path.abspath(__file__))


def _curves(name):
    d = json.load(open(os.path.join(HERE, "golden", name)))
    C = {k: np.array([c[k] for c in d["curves"]]) for k in ("S", "beta", "cv")}
    C["S"] = C["S"][:, :-1]                  # S is pinned to 0 at the top grid point
    return d, C


def _synthetic(rng, n, g, shift=0.0):
    """Replica curves like MUCA entropies: integrals of heavy-tailed (Student t, 3 dof) slopes,
    so neighbouring points are strongly correlated and single replicas are outliers."""
    return np.cumsum(rng.standard_t(3, size=(n, g)), axis=1) * 0.05 + shift


def test_p_values_are_calibrated_on_correlated_heavy_tailed_curves():
    rng = np.random.default_rng(20)
    trials, alpha = 300, 0.05
    rej = np.zeros(3)
    for t in range(trials):
        r = sc.permutation_test(_synthetic(rng, 16, 120), _synthetic(rng, 16, 120), n_perm=199,
                                seed=t)
        rej += np.array([r[s] <= alpha for s in sc.SUMMARIES])
    rate = rej / trials
    print("false-alarm rates", dict(zip(sc.SUMMARIES, rate)))
    # binomial(300, 0.05): mean 15, sd 3.8
    assert np.all(rej <= 15 + 3.5 * 3.8)


def test_coherent_offset_is_detected():
    """A shift of the whole curve by a fraction of the replica spread that no single grid point
    resolves at this sample size (per-point z about 0.6, so max |z| stays within its null range)
    is caught by the |mean z| summary."""
    rng = np.random.default_rng(21)
    A = rng.standard_t(3, size=(32, 150))
    B = rng.standard_t(3, size=(32, 150)) + 0.25
    r = sc.permutation_test(A, B, n_perm=2999)
    print({s: r[s] for s in sc.SUMMARIES})
    assert r["abs_mean_z"] < 0.001
    assert r["max_abs_z"] > 0.01


@pytest.mark.parametrize("name", ["muca_c1_reference.json", "muca_n6_reference.json"])
def test_disjoint_halves_of_oracle_replicas_pass(name):
    _, C = _curves(name)
    ok, res = sc.compare_curves({k: v[0::2] for k, v in C.items()},
                                {k: v[1::2] for k, v in C.items()})
    print({k: {s: r[s] for s in sc.SUMMARIES} for k, r in res.items()})
    assert ok


def test_random_splits_of_oracle_replicas_reject_at_the_nominal_rate():
    _, C = _curves("muca_c1_reference.json")
    S = C["S"]
    rng = np.random.default_rng(22)
    n_split = 150
    p = []
    for t in range(n_split):
        perm = rng.permutation(len(S))
        h = len(S) // 2
        p.append(sc.permutation_test(S[perm[:h]], S[perm[h:]], n_perm=499, seed=t)["max_abs_z"])
    p = np.array(p)
    print("fraction of splits with p <= 0.05:", (p <= 0.05).mean())
    # splits of one set are dependent, so this is a loose check of the nominal 5 %
    assert (p <= 0.05).mean() <= 0.15


def _planted_replica(args):
    import oracle
    import workloads
    from oracle import analysis
    r, d, k_bend = args
    wl = workloads.single_chain(n=6)
    wl.k_bend = k_bend
    sp = wl.systems[0]
    res = oracle.muca(wl, n_iter=d["iterations"], n_sweeps=d["sweeps"], walkers=d["walkers"],
                      seed=40000 + r)
    a = analysis.analyze(res["beta"], res["alpha"], sp.e_lo, wl.bin_width, d["k_lo"], d["k_hi"],
                         d["iterations"] - d["block"], d["iterations"], d["block"],
                         wl.bin_width, beta_c=1.0)
    return a["S"][:-1], a["beta"], a["cv"]


def test_planted_oracle_error_is_rejected(orc):
    """16 replicas of an oracle whose bending coupling is 0.30 instead of 0.25, at the
    schedule of the stored 6-bead reference, fail the criterion against that reference."""
    d, C = _curves("muca_n6_reference.json")
    with Pool(8) as pool:
        out = pool.map(_planted_replica, [(r, d, 0.30) for r in range(16)])
    G = {k: np.array([o[i] for o in out]) for i, k in enumerate(("S", "beta", "cv"))}
    ok, res = sc.compare_curves(G, C)
    print({k: {s: r[s] for s in sc.SUMMARIES} for k, r in res.items()})
    assert not ok
