"""Statistical parity of the GPU MUCA estimate with the FP64 oracle: replicas of S(E), the
caloric curve beta(E) and the specific heat C_V(E) (Eqs. 4-6) from independent GPU runs must be
draws from the distribution of the oracle's replicas, judged by the exactly calibrated rank
permutation test of tests/stats_criteria.py at a family-wise false-alarm level of 1 % (its
calibration, its power against a planted oracle error and its verdict on halves of the oracle's
own replicas are checked on the CPU in test_stats_criteria.py).

  * the 13-bead chain at its full budget (one walker, ten iterations of 10^5 sweeps, FP64):
    32 GPU replicas against the 32 oracle replicas of tests/golden/muca_c1_reference.json;
  * a 6-bead chain in the FP32-split precision (FP32 pair terms, FP64 resync every 100
    sweeps), four walkers sharing the weights, twelve iterations of 2 x 10^4 sweeps: 32 GPU
    replicas against tests/golden/muca_n6_reference.json.

Both reference files are written by scripts beside them that call only the oracle.  The GPU side
runs its replicas as independent systems of one context (each with its own weights, histogram
and walkers; distinct walker ids give distinct random streams, and the seed differs from every
oracle seed) and analyses them with the library's own microcanonical_analyze."""
import json
import os

import numpy as np
import pytest

import stats_criteria as sc
import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _oracle_curves(ref):
    C = {k: np.array([c[k] for c in ref["curves"]]) for k in ("S", "beta", "cv")}
    C["S"] = C["S"][:, :-1]                  # S is pinned to 0 at the top grid point
    return C


def _run_replicas(P, wl_one, R, walkers, iters, sweeps, keep_from, seed, **over):
    sp = wl_one.systems[0]
    wl_one.systems = [sp] * R
    init = [workloads.initial_positions(wl_one)[0]] * R
    m = P.Muca.from_workload(wl_one, init, walkers=walkers, seed=seed, **over)
    print("launch plan", m.launch_info(), flush=True)
    betas = [[] for _ in range(R)]
    alphas = [[] for _ in range(R)]
    for it in range(iters):
        m.iterate(sweeps, 1)
        if it >= keep_from:
            for r in range(R):
                b, a, _ = m.weights(r)
                betas[r].append(b)
                alphas[r].append(a)
        print(f"iteration {it} done", flush=True)
    m.close()
    return sp, betas, alphas


def _gpu_curves(P, sp, wl, betas, alphas, k_lo, k_hi, block, dE):
    G = {"S": [], "beta": [], "cv": []}
    for b, a in zip(betas, alphas):
        res = P.microcanonical_analyze(np.array(b), np.array(a), sp.e_lo, wl.bin_width, k_lo,
                                       k_hi, 0, block, block, dE, beta_c=1.0)
        G["S"].append(res["S"][:-1])
        G["beta"].append(res["beta"])
        G["cv"].append(res["cv"])
    return {k: np.array(v) for k, v in G.items()}


def _judge(G, C):
    ok, res = sc.compare_curves(G, C, family_alpha=0.01)
    for k, r in res.items():
        print(k, "points", r["n_points"], {s: round(float(r[s]), 4) for s in sc.SUMMARIES},
              {s: round(float(v), 3) for s, v in r["stats"].items()})
    return ok


def test_config1_fp64_replicas_match_oracle():
    import paper_1702_01770_amd as P
    ref = json.load(open(os.path.join(HERE, "golden", "muca_c1_reference.json")))
    wl = workloads.single_chain()
    R, iters, sweeps = ref["replicas"], ref["iterations"], ref["sweeps"]
    keep = ref["block_start"]
    sp, betas, alphas = _run_replicas(P, wl, R, 1, iters, sweeps, keep, seed=9_100_001,
                                      precision=0)
    G = _gpu_curves(P, sp, wl, betas, alphas, ref["k_lo"], ref["k_hi"], iters - keep, ref["dE"])
    assert _judge(G, _oracle_curves(ref))


def test_fp32_split_replicas_match_oracle():
    import paper_1702_01770_amd as P
    ref = json.load(open(os.path.join(HERE, "golden", "muca_n6_reference.json")))
    wl = workloads.single_chain(n=6)
    R, Wk, iters, sweeps, block = (ref["replicas"], ref["walkers"], ref["iterations"],
                                   ref["sweeps"], ref["block"])
    sp, betas, alphas = _run_replicas(P, wl, R, Wk, iters, sweeps, iters - block,
                                      seed=9_000_001, precision=1, resync_sweeps=100)
    G = _gpu_curves(P, sp, wl, betas, alphas, ref["k_lo"], ref["k_hi"], block, wl.bin_width)
    assert _judge(G, _oracle_curves(ref))
