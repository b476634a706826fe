"""End-to-end FP64 parity of the captured MUCA iteration loop (muca_iterate: sweep launches plus
the weight update in one HIP graph, Sec. 2.2, Fig. 2) against the oracle's serial parallel-MUCA
scheme, on runs whose sweeps per iteration exceed one launch, so that every walker crosses
launch boundaries inside each iteration; and of the accept log over launch boundaries and over
successive muca_sweep calls."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1702_01770_amd as P
    P.load()
    return P


def _oracle_runs(orc, wl, systems, walkers, n_iter, n_sweeps):
    return {s: orc.muca(wl, s, n_iter=n_iter, n_sweeps=n_sweeps, walkers=walkers,
                        walker_offset=s * walkers) for s in systems}


def _check_final_state(m, orc, wl, s, res, walkers, n_iter, n_sweeps):
    b, a, g = m.weights(s)
    W = res["weights"]
    assert np.allclose(b, W.beta, rtol=1e-12, atol=1e-12), f"system {s}: beta"
    assert np.allclose(a, W.alpha, rtol=1e-12, atol=1e-9), f"system {s}: alpha"
    assert np.allclose(g, W.g, rtol=1e-12, atol=0), f"system {s}: g"
    assert np.array_equal(m.histogram(s, last=True), res["hist"][-1]), f"system {s}: last H"
    assert not m.histogram(s).any()                  # the update cleared the running one
    pos_g, e_g, cnt = m.walkers_state(s)
    sysd = orc.System.from_workload(wl, s)
    for i, ow in enumerate(res["walkers"]):
        _, _, scale = sysd.energy_parts(ow.pos)
        assert np.allclose(pos_g[i], ow.pos, rtol=0, atol=1e-10), f"system {s} walker {i}"
        assert e_g[i] == pytest.approx(ow.energy, abs=1e-11 * max(1.0, scale))
        assert cnt["moves"][i] == ow.counters.moves
        assert cnt["accepted"][i] == ow.counters.accepted
        assert cnt["window_rejects"][i] == ow.counters.window_rejects
        assert cnt["sweeps"][i] == n_iter * n_sweeps


def _check_stats(m, s, res, n_iter, n_sys):
    st = m.stats_history(0, n_iter)
    for it in range(n_iter):
        H = res["hist"][it]
        cv, pk, lo, hi = res["flat"][it]
        moves, cvar, peak, kmin, kmax = st[it, s]
        assert moves == int(H.sum()), (s, it)
        assert (kmin, kmax) == (lo, hi), (s, it)
        assert cvar == pytest.approx(cv, rel=1e-12), (s, it)
        assert peak == pytest.approx(pk, rel=1e-12), (s, it)


@pytest.mark.parametrize("pack", [1, 2])
def test_iterate_matches_oracle_across_launches(lib, orc, pack):
    """Chains of 13, 24 and 100 beads: the 100-bead chain sets 2000 sweeps per launch, so each
    iteration of 2500 sweeps is two launches for every walker.  One muca_iterate call of three
    iterations is compared at the end (weights, statistics of every iteration, last histogram,
    walkers); a second context runs one iteration per call and its histogram of every iteration
    is compared bit for bit."""
    wl = workloads.chains_of_lengths([13, 24, 100], walkers=2)
    n_iter, n_sweeps, walkers = 3, 2500, 2
    systems = list(range(wl.n_systems))
    res = _oracle_runs(orc, wl, systems, walkers, n_iter, n_sweeps)
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=walkers, precision=0,
                               walkers_per_wave=pack)
    info = m.launch_info()
    print("launch plan", info)
    assert info["sweeps_per_launch"] < n_sweeps
    m.iterate(n_sweeps, n_iter)
    for s in systems:
        _check_final_state(m, orc, wl, s, res[s], walkers, n_iter, n_sweeps)
        _check_stats(m, s, res[s], n_iter, wl.n_systems)
    m.close()
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=walkers, precision=0,
                               walkers_per_wave=pack)
    for it in range(n_iter):
        m.iterate(n_sweeps, 1)
        for s in systems:
            assert np.array_equal(m.histogram(s, last=True), res[s]["hist"][it]), (s, it)
            b, _, _ = m.weights(s)
            assert np.allclose(b, res[s]["beta"][it], rtol=1e-12, atol=1e-12), (s, it)
    m.close()


def test_iterate_mixed_plan_sampled_systems(lib, orc):
    """The batched workload's 32 systems (13..55 beads) in the mixed launch plan (16-, 32- and
    64-lane walkers in one launch), 16 walkers per system, FP64, two iterations of 4000 sweeps
    (3636 per launch).  The shortest, the longest and a middle system are run by the oracle with
    all of their walkers and compared after the captured loop."""
    wl = workloads.batched_chains(walkers=512, precision=0)
    n_iter, n_sweeps, walkers = 2, 4000, 16
    lens = [sp.n_beads for sp in wl.systems]
    order = np.argsort(lens, kind="stable")
    systems = sorted({int(order[0]), int(order[len(order) // 2]), int(order[-1])})
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=walkers, precision=0,
                               walkers_per_wave=-1)
    info = m.launch_info()
    print("launch plan", info, "systems", systems, [lens[s] for s in systems])
    assert info["walkers_per_wave"] == -1 and info["sweeps_per_launch"] < n_sweeps
    assert info["lanes_used"] & 0b100
    m.iterate(n_sweeps, n_iter)
    res = _oracle_runs(orc, wl, systems, walkers, n_iter, n_sweeps)
    for s in systems:
        _check_final_state(m, orc, wl, s, res[s], walkers, n_iter, n_sweeps)
        _check_stats(m, s, res[s], n_iter, wl.n_systems)
    m.close()


@pytest.mark.parametrize("pack", [1, 2])
def test_accept_log_spans_launches_and_calls(lib, orc, pack):
    """One accept log armed before two muca_sweep calls, the first of which is two launches
    (2500 sweeps at 2000 per launch): bit i of a walker is its i-th single-bead move since the
    log was armed, whichever launch or call made it."""
    wl = workloads.chains_of_lengths([13, 100], walkers=2)
    walkers = 2
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=walkers, precision=0,
                               walkers_per_wave=pack)
    assert m.launch_info()["sweeps_per_launch"] == 2000
    m.sweep(100)                                    # the log starts after some moves were made
    first, second = 2500, 300
    n_log = (first + second) * 13 + 500             # the 13-bead chain fills all but the tail
    m.set_accept_log(n_log)
    m.sweep(first)
    m.sweep(second)
    for s in range(wl.n_systems):
        sp = wl.systems[s]
        sysd = orc.System.from_workload(wl, s)
        W = orc.Weights(sp.e_lo, wl.bin_width, sp.n_bins)
        log_g = m.accept_log(s)
        pos_g, _, cnt = m.walkers_state(s)
        for i in range(walkers):
            ow = orc.Walker(sysd, workloads.initial_positions(wl)[s], s * walkers + i, wl.seed)
            ow.run(W, orc.move_params(wl), 100, np.zeros(sp.n_bins, np.uint64))
            log = np.zeros(n_log, np.uint8)
            ow.run(W, orc.move_params(wl), first + second, np.zeros(sp.n_bins, np.uint64),
                   accept_log=log)
            assert np.array_equal(log_g[i], log), f"system {s} walker {i}"
            assert log.sum() > 0
            assert np.allclose(pos_g[i], ow.pos, rtol=0, atol=1e-10)
            assert cnt["moves"][i] == ow.counters.moves
    m.close()
