"""Write tests/golden/muca_c1_reference.json: the FP64 oracle's MUCA estimate for the single
13-bead chain (workloads.single_chain(): one walker, ten iterations of 10^5 sweeps, bins of 0.05
in [-52, 13)) from independent replicas, and a longer parallel-MUCA reference of its entropy.

Calls only oracle/ and workloads/ (independent processes, one replica each).

  replicas  REPLICAS runs at exactly that budget (seeds SEED0 + r, walker 0).  For each, the
            microcanonical analysis (Eqs. 4-6, oracle.analysis) of its last two iterations as
            one block on the centres of bins [K_LO, K_HI) with difference step DE: S(E)
            (normalised to 0 at the top grid point), beta(E), C_V(E).  These are the samples of
            the statistical parity test.
  reference REF_RUNS parallel-MUCA runs (Sec. 2.2: REF_WALKERS walkers sharing the weights,
            REF_ITERS iterations of REF_SWEEPS sweeps per walker; seeds REF_SEED0 + 1000 r).
            S_ref is the mean over runs of the entropy of their last weights, S_n(E) =
            beta_k E - alpha_k at the grid points, with its standard error.  Below about
            E = -7 neither these runs nor the replicas converge (walkers freeze in compact
            states where the recursion's low-energy slopes trap them); the "converged" range is
            the top part of the grid where the replicas agree to better than SIGMA_CONV and the
            reference's standard error is below 0.3 of the replicas' spread.
  target    the matched-error target of the benchmark: the aligned error of a replica at the
            budget, delta_S = max over converged bins |S_10 - S_ref - c| (c the offset that
            minimises the sum of ((S_10 - S_ref - c) / sigma_k)^2, sigma_k the replicas'
            spread; the top point, where every S is pinned to 0, left out), as the median over
            replicas.
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402
from oracle import analysis  # noqa: E402

REPLICAS, ITERS, SWEEPS, SEED0 = 32, 10, 100000, 7000
BLOCK_START = 8                       # iterations [8, 10) form the analysed block
K_LO, K_HI = 700, 1290
DE = 0.2                              # 4 bins
REF_RUNS, REF_WALKERS, REF_SWEEPS, REF_ITERS, REF_SEED0 = 16, 32, 5000, 30, 90000
SIGMA_CONV = 0.1


def _grid_entropy(beta, alpha, e_lo, eps):
    E = e_lo + (np.arange(K_LO, K_HI) + 0.5) * eps
    S = analysis.s_of_e(beta, alpha, e_lo, eps, E)
    return S - S[..., -1:]


def replica(r):
    wl = workloads.single_chain()
    sp = wl.systems[0]
    res = oracle.muca(wl, n_iter=ITERS, n_sweeps=SWEEPS, walkers=1, seed=SEED0 + r)
    a = analysis.analyze(res["beta"], res["alpha"], sp.e_lo, wl.bin_width, K_LO, K_HI,
                         BLOCK_START, ITERS, ITERS - BLOCK_START, DE, beta_c=1.0)
    s_last = _grid_entropy(res["beta"][-1], res["alpha"][-1], sp.e_lo, wl.bin_width)
    return dict(S=a["S"], beta=a["beta"], cv=a["cv"], S_last=s_last)


def reference_run(r):
    wl = workloads.single_chain()
    sp = wl.systems[0]
    res = oracle.muca(wl, n_iter=REF_ITERS, n_sweeps=REF_SWEEPS, walkers=REF_WALKERS,
                      seed=REF_SEED0 + 1000 * r)
    return _grid_entropy(res["beta"][-1], res["alpha"][-1], sp.e_lo, wl.bin_width)


def aligned_error(S, S_ref, sigma, sl):
    d = S[sl] - S_ref[sl]
    w = 1.0 / sigma[sl] ** 2
    c = np.sum(w * d) / np.sum(w)
    return float(np.max(np.abs(d - c)))


def _r(a, digits=9):
    return [float(f"{x:.{digits}g}") for x in np.asarray(a, dtype=np.float64)]


def main():
    wl = workloads.single_chain()
    sp = wl.systems[0]
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        reps = pool.map(replica, range(REPLICAS))
        refs = np.array(pool.map(reference_run, range(REF_RUNS)))
    S_ref = refs.mean(axis=0)
    se_ref = refs.std(axis=0, ddof=1) / np.sqrt(REF_RUNS)
    S_last = np.array([r["S_last"] for r in reps])
    sigma = S_last.std(axis=0, ddof=1)
    # converged: the replicas agree to better than SIGMA_CONV and the reference is at least
    # ~3x more precise than one replica (the top point, where S is pinned to 0, is left out)
    ok = (sigma < SIGMA_CONV) & (se_ref < 0.3 * sigma)
    k = len(ok) - 1
    while k > 0 and ok[k - 1]:
        k -= 1
    conv_lo = k                        # grid index where the converged top range starts
    sl = slice(conv_lo, len(ok) - 1)
    deltas = [aligned_error(s, S_ref, sigma, sl) for s in S_last]
    out = dict(workload="single_chain(seed=1702, n=13)", replicas=REPLICAS, walkers=1,
               iterations=ITERS, sweeps=SWEEPS, seed0=SEED0, block_start=BLOCK_START,
               k_lo=K_LO, k_hi=K_HI, dE=DE, e_lo=sp.e_lo, bin_width=wl.bin_width,
               curves=[dict(S=_r(r["S"]), beta=_r(r["beta"]), cv=_r(r["cv"])) for r in reps],
               reference=dict(runs=REF_RUNS, walkers=REF_WALKERS, sweeps=REF_SWEEPS,
                              iterations=REF_ITERS, seed0=REF_SEED0, S=_r(S_ref),
                              se=_r(se_ref), replica_sigma=_r(sigma),
                              converged_from=int(conv_lo), sigma_conv=SIGMA_CONV,
                              converged_e=float(sp.e_lo + (K_LO + conv_lo + 0.5) * wl.bin_width)),
               target=dict(replica_delta_S=_r(deltas), delta_S=float(np.median(deltas))))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "muca_c1_reference.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", path, "converged from grid index", conv_lo, "E =",
          out["reference"]["converged_e"], "target delta_S", out["target"]["delta_S"])


if __name__ == "__main__":
    main()
