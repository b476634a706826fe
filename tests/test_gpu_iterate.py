"""FP64 parity of the captured MUCA iteration loop (muca_iterate: the sweep launches plus the
weight update of Sec. 2.2 / Fig. 2 in one HIP graph) with the oracle, on iterations whose sweeps
exceed one launch, so that every walker crosses launch boundaries inside each iteration; and of
the accept log over launch boundaries and successive muca_sweep calls.

FP64 trajectories of the two implementations agree move for move as long as their running
energies agree to rounding; the two sum the pair terms in different orders, so over many MUCA
iterations (which drive walkers into states with large, cancelling pair terms) the rounding
difference eventually flips a near-tie and the chains part.  The loop is therefore compared one
iteration at a time: before each iteration the oracle walkers take over the GPU's coordinates,
running energies and stream positions and the oracle takes the GPU's weights; then the
iteration's histogram (bit for bit), the updated weights, the statistics, the walkers'
coordinates, energies and counters must agree.  The windows end at E = +1 (instead of +N) so
that walkers stay out of overlapping states whose pair terms would amplify rounding.  Separately,
one muca_iterate call of several iterations must reproduce the GPU's own iteration-by-iteration
run bit for bit (the graph replays are the stepwise loop)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1702_01770_amd as P
    P.load()
    return P


def _narrow(wl):
    """Window [-4N, +1) for every system."""
    for sp in wl.systems:
        sp.n_bins = int(round((4.0 * sp.n_beads + 1.0) / wl.bin_width))
    return wl


def _resync_iteration(m, orc, wl, systems, walkers, n_sweeps):
    """Oracle iteration started from the GPU's state and weights; runs the GPU iteration too."""
    before = {s: (m.walkers_state(s), m.weights(s)) for s in systems}
    m.iterate(n_sweeps, 1)
    out = {}
    mv = orc.move_params(wl)
    for s in systems:
        sp = wl.systems[s]
        sysd = orc.System.from_workload(wl, s)
        (pos0, e0, c0), (b, a, g) = before[s]
        W = orc.Weights(sp.e_lo, wl.bin_width, sp.n_bins, b, a, g)
        H = np.zeros(sp.n_bins, np.uint64)
        ws = []
        for i in range(walkers):
            w = orc.Walker(sysd, pos0[i], s * walkers + i, wl.seed)
            w.energy = float(e0[i])                   # the GPU's running energy, not a recompute
            w.sweeps = int(c0["sweeps"][i])
            w.run(W, mv, n_sweeps, H)
            ws.append((w, c0))
        W.berg_update(H)
        out[s] = (H, W, ws)
    return out


def _check_iteration(m, orc, wl, it, res, n_sweeps):
    st = m.stats_history(it, 1)
    for s, (H, W, ws) in res.items():
        assert np.array_equal(m.histogram(s, last=True), H), f"iteration {it} system {s}: H"
        assert not m.histogram(s).any()
        b, a, g = m.weights(s)
        assert np.allclose(b, W.beta, rtol=1e-12, atol=1e-12), (it, s, "beta")
        assert np.allclose(a, W.alpha, rtol=1e-12, atol=1e-9), (it, s, "alpha")
        assert np.allclose(g, W.g, rtol=1e-12, atol=0), (it, s, "g")
        cv, pk, lo, hi = orc.flatness(H)
        moves, cvar, peak, kmin, kmax = st[0, s]
        assert moves == int(H.sum()) and (kmin, kmax) == (lo, hi), (it, s)
        assert cvar == pytest.approx(cv, rel=1e-12) and peak == pytest.approx(pk, rel=1e-12)
        pos_g, e_g, cnt = m.walkers_state(s)
        sysd = orc.System.from_workload(wl, s)
        for i, (w, c0) in enumerate(ws):
            # every decision is identical (counters, histogram); coordinates and running
            # energies carry the rounding of 10^5 moves, which folded chains amplify (the
            # crankshaft axis of a sharply bent bead is short), hence the looser bounds
            _, _, scale = sysd.energy_parts(w.pos)
            assert np.allclose(pos_g[i], w.pos, rtol=0, atol=1e-7), (it, s, i)
            assert e_g[i] == pytest.approx(w.energy, abs=1e-9 * max(1.0, scale)), (it, s, i)
            assert cnt["moves"][i] - c0["moves"][i] == w.counters.moves
            assert cnt["accepted"][i] - c0["accepted"][i] == w.counters.accepted
            assert cnt["window_rejects"][i] - c0["window_rejects"][i] == w.counters.window_rejects
            assert cnt["sweeps"][i] == c0["sweeps"][i] + n_sweeps


@pytest.mark.parametrize("pack", [1, 2])
def test_iterate_matches_oracle_iteration_by_iteration(lib, orc, pack):
    """Chains of 13, 24 and 64 beads, two walkers each: the 64-bead chain sets 3125 sweeps per
    launch, so each iteration of 3500 sweeps is two launches for every walker (one walker per
    wave: one system per workgroup, whose ln W table must fit in LDS)."""
    wl = _narrow(workloads.chains_of_lengths([13, 24, 64], walkers=2))
    n_iter, n_sweeps, walkers = 3, 3500, 2
    kw = dict(walkers_per_wave=pack, waves_per_block=2 if pack == 1 else 0)
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=walkers, precision=0,
                               **kw)
    info = m.launch_info()
    print("launch plan", info)
    assert info["sweeps_per_launch"] < n_sweeps < 2 * info["sweeps_per_launch"]
    for it in range(n_iter):
        res = _resync_iteration(m, orc, wl, range(wl.n_systems), walkers, n_sweeps)
        _check_iteration(m, orc, wl, it, res, n_sweeps)
    m.close()


def test_iterate_mixed_plan_sampled_systems(lib, orc):
    """The batched workload's 32 systems (13..55 beads) in the mixed launch plan (16-, 32- and
    64-lane walkers in one launch), 16 walkers per system, FP64, iterations of 4000 sweeps
    (3636 per launch).  The shortest, a middle and the longest system are followed by the oracle
    with all of their walkers, iteration by iteration."""
    wl = _narrow(workloads.batched_chains(walkers=512, precision=0))
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
    for it in range(n_iter):
        res = _resync_iteration(m, orc, wl, systems, walkers, n_sweeps)
        _check_iteration(m, orc, wl, it, res, n_sweeps)
    m.close()


def test_one_iterate_call_equals_the_stepwise_loop(lib):
    """muca_iterate(n, 4) (one graph, replayed four times) against four muca_sweep(n) +
    muca_update_weights calls on a second context: identical histograms, weights, walkers and
    statistics, with the default windows and launches split inside each iteration."""
    wl = workloads.chains_of_lengths([13, 24, 64], walkers=4)
    n_sweeps, n_iter = 3500, 4
    a = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=4, precision=0)
    b = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=4, precision=0)
    a.iterate(n_sweeps, n_iter)
    for _ in range(n_iter):
        b.sweep(n_sweeps)
        b.update_weights()
    assert np.array_equal(a.stats_history(0, n_iter), b.stats_history(0, n_iter))
    for s in range(wl.n_systems):
        assert np.array_equal(a.histogram(s, last=True), b.histogram(s, last=True))
        for x, y in zip(a.weights(s), b.weights(s)):
            assert np.array_equal(x, y)
        pa, ea, ca = a.walkers_state(s)
        pb, eb, cb = b.walkers_state(s)
        assert np.array_equal(pa, pb) and np.array_equal(ea, eb)
        for k in ca:
            assert np.array_equal(ca[k], cb[k]), k
    a.close()
    b.close()


@pytest.mark.parametrize("pack", [1, 2])
def test_accept_log_spans_launches_and_calls(lib, orc, pack):
    """One accept log armed before two muca_sweep calls, the first of which is two launches
    (3500 sweeps at 3125 per launch): bit i of a walker is its i-th single-bead move since the
    log was armed, whichever launch or call made it."""
    wl = workloads.chains_of_lengths([13, 64], walkers=2)
    walkers = 2
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=walkers, precision=0,
                               walkers_per_wave=pack, waves_per_block=2 if pack == 1 else 0)
    assert m.launch_info()["sweeps_per_launch"] == 3125
    m.sweep(100)                                    # the log starts after some moves were made
    first, second = 3500, 300
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
            # identical decisions; coordinates carry the rounding of 2.5 x 10^5 moves of a
            # 64-bead chain (about 2e-7 here, on coordinates of size ~50)
            assert np.allclose(pos_g[i], ow.pos, rtol=0, atol=1e-6)
            assert cnt["moves"][i] == ow.counters.moves
    m.close()
