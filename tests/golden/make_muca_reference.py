"""Write tests/golden/muca_n6_reference.json: per-replica microcanonical curves S(E), beta(E),
C_V(E) of the FP64 oracle's MUCA estimate for a 6-bead chain (workloads.single_chain(n=6)),
short enough for the recursion to flatten the histogram within a dozen iterations.

Calls only oracle/ and workloads/.  Schedule: REPLICAS independent seeds, each running the
parallel MUCA scheme of Sec. 2.2 with WALKERS walkers for ITERS iterations of SWEEPS sweeps;
the analysis (Eqs. 4-6, oracle.analysis) averages the last BLOCK iterations on the centres of
bins [K_LO, K_HI) (chosen inside the range every replica visited in its last iteration).
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402
from oracle import analysis  # noqa: E402

REPLICAS, WALKERS, ITERS, SWEEPS, BLOCK = 32, 4, 12, 20000, 4
SEED0 = 500


def main():
    wl = workloads.single_chain(n=6)
    sp = wl.systems[0]
    runs = [oracle.muca(wl, n_iter=ITERS, n_sweeps=SWEEPS, walkers=WALKERS, seed=SEED0 + r)
            for r in range(REPLICAS)]
    lo = max(int(np.nonzero(r["hist"][-1])[0][0]) for r in runs)
    hi = min(int(np.nonzero(r["hist"][-1])[0][-1]) for r in runs)
    k_lo, k_hi = lo + 4, hi - 4
    curves = []
    for r in runs:
        a = analysis.analyze(r["beta"], r["alpha"], sp.e_lo, wl.bin_width, k_lo, k_hi,
                             ITERS - BLOCK, ITERS, BLOCK, wl.bin_width, beta_c=1.0)
        curves.append(dict(S=a["S"].tolist(), beta=a["beta"].tolist(), cv=a["cv"].tolist()))
    out = dict(workload="single_chain(seed=1702, n=6)", replicas=REPLICAS, walkers=WALKERS,
               iterations=ITERS, sweeps=SWEEPS, block=BLOCK, seed0=SEED0, k_lo=k_lo, k_hi=k_hi,
               e_lo=sp.e_lo, bin_width=wl.bin_width, curves=curves)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "muca_n6_reference.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path, "grid", k_lo, k_hi)


if __name__ == "__main__":
    main()
