"""Statistical parity of the GPU MUCA estimate (FP32 pair terms, FP64 resync every 100 sweeps)
with the FP64 oracle: S(E) and the caloric curve beta(E) from independent replicas must agree
within their combined standard errors.  The oracle replicas are stored in
tests/golden/muca_n6_reference.json (written by tests/golden/make_muca_reference.py, which calls
only the oracle).

The z-scores of neighbouring grid points are strongly correlated (S is an integral of beta), so
a whole curve can sit one or two standard errors off by chance; the test bounds the largest |z|
over the grid and the grid-averaged z (whose standard deviation is at most 1 under the null)."""
import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_gpu_replicas_match_oracle_entropy_and_caloric_curve():
    import paper_1702_01770_amd as P
    ref = json.load(open(os.path.join(HERE, "golden", "muca_n6_reference.json")))
    R, Wk, iters, sweeps, block = (ref["replicas"], ref["walkers"], ref["iterations"],
                                   ref["sweeps"], ref["block"])
    k_lo, k_hi = ref["k_lo"], ref["k_hi"]
    wl = workloads.single_chain(n=6)
    sp = wl.systems[0]
    # R independent MUCA runs at once: R copies of the system, each with its own weights,
    # histogram and walkers (distinct walker ids give distinct random streams)
    wl.systems = [sp] * R
    init = [workloads.initial_positions(workloads.single_chain(n=6))[0]] * R
    m = P.Muca.from_workload(wl, init, walkers=Wk, precision=1, seed=9_000_001,
                             resync_sweeps=100)
    betas = [[] for _ in range(R)]
    alphas = [[] for _ in range(R)]
    for it in range(iters):
        m.sweep(sweeps)
        m.update_weights()
        for r in range(R):
            b, a, _ = m.weights(r)
            betas[r].append(b)
            alphas[r].append(a)
    m.close()
    gS, gB = [], []
    for r in range(R):
        res = P.microcanonical_analyze(np.array(betas[r]), np.array(alphas[r]), sp.e_lo,
                                       wl.bin_width, k_lo, k_hi, iters - block, iters, block,
                                       wl.bin_width, beta_c=1.0)
        gS.append(res["S"])
        gB.append(res["beta"])
    gS, gB = np.array(gS), np.array(gB)
    oS = np.array([c["S"] for c in ref["curves"]])
    oB = np.array([c["beta"] for c in ref["curves"]])

    def z(g, o):
        se = np.sqrt(g.var(axis=0, ddof=1) / len(g) + o.var(axis=0, ddof=1) / len(o))
        return (g.mean(axis=0) - o.mean(axis=0)) / np.maximum(se, 1e-12)

    zs, zb = z(gS[:, :-1], oS[:, :-1]), z(gB, oB)      # S is pinned to 0 at the top point
    print("max |z| S:", np.abs(zs).max(), " beta:", np.abs(zb).max(),
          " mean z S:", zs.mean(), " beta:", zb.mean())
    assert np.abs(zs).max() < 5.0
    assert np.abs(zb).max() < 5.0
    assert abs(zs.mean()) < 3.0 and abs(zb.mean()) < 3.0
