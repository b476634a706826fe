"""GPU parity of the MUCA sweep and weight update against the FP64 oracle, through the C ABI.

FP64 mode: the same Philox streams give the same trajectories, so accept/reject sequences and
histogram counts must agree bit for bit, coordinates and energies to rounding (1e-11 relative to
the energy scale).  FP32-split mode: pair terms in FP32, so trajectories differ; the running
energy of each walker must stay within 1e-5 of the sum of term magnitudes of the FP64 energy of
its own coordinates."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1702_01770_amd as P
    P.load()
    return P


def _oracle_walkers(orc, wl, sys_index, walkers, n_sweeps, weights=None, log_moves=0,
                    first_walker=None):
    sp = wl.systems[sys_index]
    s = orc.System.from_workload(wl, sys_index)
    pos0 = workloads.initial_positions(wl)[sys_index]
    W = weights if weights is not None else orc.Weights(sp.e_lo, wl.bin_width, sp.n_bins)
    H = np.zeros(sp.n_bins, np.uint64)
    out = []
    base = sys_index * walkers if first_walker is None else first_walker
    for i in range(walkers):
        w = orc.Walker(s, pos0, base + i, wl.seed)
        log = np.zeros(log_moves, np.uint8) if log_moves else None
        w.run(W, orc.move_params(wl), n_sweeps, H, accept_log=log)
        out.append((w, log))
    return H, out


def _compare(lib, orc, wl, walkers, n_sweeps, weights_by_sys=None, log_moves=None, pack=1,
             **over):
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=walkers, precision=0,
                               walkers_per_wave=pack, **over)
    info = m.launch_info()
    assert info["walkers_per_wave"] == pack
    print("launch plan", info)
    if weights_by_sys:
        for s, Wt in weights_by_sys.items():
            m.set_weights(s, Wt.beta, Wt.alpha, Wt.g)
    n_log = log_moves if log_moves is not None else n_sweeps * min(x.n_beads for x in wl.systems)
    m.set_accept_log(n_log)
    m.sweep(n_sweeps)
    for s in range(wl.n_systems):
        sp = wl.systems[s]
        Wt = weights_by_sys.get(s) if weights_by_sys else None
        H, ows = _oracle_walkers(orc, wl, s, walkers, n_sweeps, Wt, log_moves=n_log)
        Hg = m.histogram(s)
        log_g = m.accept_log(s)
        pos_g, e_g, cnt = m.walkers_state(s)
        print(f"system {s}: N={sp.n_beads} moves={int(H.sum())}")
        assert np.array_equal(Hg, H), "histograms differ"
        for i, (ow, olog) in enumerate(ows):
            assert np.array_equal(log_g[i], olog), f"accept sequence of walker {i} differs"
            _, _, scale = orc.System.from_workload(wl, s).energy_parts(ow.pos)
            assert np.allclose(pos_g[i], ow.pos, rtol=0, atol=1e-10)
            assert e_g[i] == pytest.approx(ow.energy, abs=1e-11 * max(1.0, scale))
            assert cnt["moves"][i] == ow.counters.moves
            assert cnt["accepted"][i] == ow.counters.accepted
            assert cnt["rigid_moves"][i] == ow.counters.rigid_moves
            assert cnt["rigid_accepted"][i] == ow.counters.rigid_accepted
            assert cnt["window_rejects"][i] == ow.counters.window_rejects
            assert cnt["pivot_moves"][i] == ow.counters.pivot_moves
            assert cnt["pivot_accepted"][i] == ow.counters.pivot_accepted
            assert cnt["rot_moves"][i] == ow.counters.rot_moves
            assert cnt["rot_accepted"][i] == ow.counters.rot_accepted
            assert cnt["sweeps"][i] == n_sweeps
    m.close()


def _walkers(pack, at_least):
    """Smallest multiple of pack that is >= at_least."""
    return -(-at_least // pack) * pack


# pack = walkers per wavefront: 1 runs k_sweep; 2 and 4 run k_sweep_pair with groups of 32 and 16
# lanes per walker
@pytest.mark.parametrize("pack", [1, 2, 4])
def test_fp64_single_chain_flat_weights(lib, orc, pack):
    wl = workloads.single_chain()
    _compare(lib, orc, wl, walkers=pack, n_sweeps=3000, pack=pack)


@pytest.mark.parametrize("pack", [1, 2, 4])
def test_fp64_single_chain_muca_weights_several_walkers(lib, orc, pack):
    wl = workloads.single_chain()
    res = orc.muca(wl, n_iter=4, n_sweeps=4000, walkers=2)
    _compare(lib, orc, wl, walkers=_walkers(pack, 6), n_sweeps=1500,
             weights_by_sys={0: res["weights"]}, pack=pack)


@pytest.mark.parametrize("pack", [1, 2, 4])
def test_fp64_batched_uneven_lengths(lib, orc, pack):
    wl = workloads.batched_chains(n_seq=3, n_min=13, n_max=60)
    _compare(lib, orc, wl, walkers=_walkers(pack, 3), n_sweeps=300, pack=pack)


@pytest.mark.parametrize("pack", [1, 2, 4])
def test_fp64_batched_paired_workgroups(lib, orc, pack):
    """Long and short systems sharing workgroups (8 waves: half run the longest remaining
    system, half the shortest), with a ragged last workgroup per system."""
    wl = workloads.batched_chains(n_seq=3, n_min=13, n_max=60)
    _compare(lib, orc, wl, walkers=_walkers(pack, 18), n_sweeps=60, pack=pack,
             waves_per_block=8)


@pytest.mark.parametrize("pack", [1, 2, 4])
def test_fp64_aggregation_periodic_rigid(lib, orc, pack):
    wl = workloads.aggregation()
    _compare(lib, orc, wl, walkers=_walkers(pack, 3), n_sweeps=400, pack=pack)


@pytest.mark.parametrize("pack", [1, 2])
def test_fp64_cross_seeding_two_slots_torsion(lib, orc, pack):
    wl = workloads.cross_seeding()
    _compare(lib, orc, wl, walkers=2, n_sweeps=200, pack=pack)


@pytest.mark.parametrize("pack", [1, 2, 4])
def test_fp64_steric_sphere(lib, orc, pack):
    """The paper's container: two 9-bead chains in a sphere of radius 6 (rigid translations too)
    and a 13-bead chain in a sphere of radius 6.5; moves leaving the sphere are rejected on both
    sides, move for move."""
    import dataclasses
    wl = workloads.confined(radius=6.0)
    _compare(lib, orc, wl, walkers=_walkers(pack, 3), n_sweeps=500, pack=pack)
    wl = dataclasses.replace(workloads.single_chain(), box_kind=workloads.BOX_SPHERE, box_len=6.5)
    _compare(lib, orc, wl, walkers=_walkers(pack, 2), n_sweeps=1500, pack=pack)


@pytest.mark.parametrize("pack", [2, 4])
def test_fp64_pivots(lib, orc, pack):
    """Pivots (the beads on one side of a random bead turn about it) after every sweep of a
    13-bead chain: accept sequence, counters and coordinates match the oracle."""
    import dataclasses
    wl = dataclasses.replace(workloads.single_chain(), pivot_per_sweep=2)
    _compare(lib, orc, wl, walkers=_walkers(pack, 4), n_sweeps=800, pack=pack)


@pytest.mark.parametrize("make", [
    lambda: workloads.aggregation(),                                    # periodic, 4 x 9
    lambda: workloads.confined(radius=6.0),                            # steric sphere
    lambda: workloads.cross_seeding()])                                 # 76 beads, torsion
def test_fp64_pivots_and_chain_rotations(lib, orc, make):
    import dataclasses
    wl = dataclasses.replace(make(), pivot_per_sweep=1, rotate_per_sweep=1)
    _compare(lib, orc, wl, walkers=2, n_sweeps=200, pack=2)


@pytest.mark.parametrize("name,pack", [("abeta_dimer", 2), ("cross_human", 4), ("cross_rat", 2)])
def test_fp64_paper_systems(lib, orc, name, pack):
    """The A/B strings the paper prints for its examples, in its steric spheres, with single-bead
    moves, rigid translations, pivots and chain rotations: accept sequences, histograms,
    counters and coordinates match the oracle."""
    wl = workloads.paper_system(name, walkers=4)
    _compare(lib, orc, wl, walkers=_walkers(pack, 4), n_sweeps=300, pack=pack)


# Mixed plan (walkers_per_wave = -1): per system 16 lanes per walker (N <= 16, or short chains
# moved there to make room), 32, or a whole wave for the longest chains (N >= 0.8 N_max);
# launch_info()["lanes_used"] has bit 0, 1, 2 for 16, 32, 64 lanes.
@pytest.mark.parametrize("make,lanes", [
    (lambda: workloads.chains_of_lengths([12, 24, 40, 56]), 0b111),      # all three kinds
    (lambda: workloads.chains_of_lengths([64, 3, 33]), 0b111),           # extremes, ragged slots
    (lambda: workloads.aggregation(), 0b100),                            # periodic, rigid moves
])
def test_fp64_mixed_plan(lib, orc, make, lanes):
    wl = make()
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=4, precision=0,
                               walkers_per_wave=-1)
    assert m.launch_info()["lanes_used"] == lanes
    m.close()
    _compare(lib, orc, wl, walkers=8, n_sweeps=300, pack=-1)


def test_fp64_mixed_plan_in_blocks_of_four_waves(lib, orc):
    """The mixed plan in workgroups of four waves (one walker per wave for the 36-bead aggregate,
    so that 1024 such walkers occupy every compute unit at one wave per SIMD): the same
    trajectories as the reference, and the block size as asked."""
    wl = workloads.aggregation()
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=8, precision=0,
                               walkers_per_wave=-1, waves_per_block=4)
    info = m.launch_info()
    assert info["waves_per_block"] == 4 and info["lanes_used"] == 0b100, info
    assert info["workgroups"] == 2, info
    m.close()
    _compare(lib, orc, wl, walkers=8, n_sweeps=300, pack=-1, waves_per_block=4)


def test_fp64_mixed_plan_chain_moves(lib, orc):
    """The human cross-seeding mixture (38 beads, one walker per wave) in its sphere with
    rigid translations, pivots and chain rotations."""
    wl = workloads.paper_system("cross_human", walkers=4)
    _compare(lib, orc, wl, walkers=4, n_sweeps=200, pack=-1)


def test_mixed_plan_limits(lib):
    """The mixed plan needs walkers per system in multiples of 4, at most 64 beads, and a chain
    long enough to gain from a whole wave."""
    for wl, kw in ((workloads.single_chain(), dict(walkers=6)),              # 6 % 4 != 0
                   (workloads.cross_seeding(walkers=4), dict(walkers=4)),     # 76 beads
                   (workloads.chains_of_lengths([12, 16]), dict(walkers=4))):  # all short
        with pytest.raises(lib.MucaError) as ei:
            lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers_per_wave=-1, **kw)
        assert "INVAL" in str(ei.value)


def test_chain_moves_need_several_walkers_per_wave(lib):
    import dataclasses
    wl = dataclasses.replace(workloads.single_chain(), pivot_per_sweep=1)
    for kw in (dict(walkers=3), dict(walkers=2, walkers_per_wave=1)):
        with pytest.raises(lib.MucaError) as ei:
            lib.Muca.from_workload(wl, workloads.initial_positions(wl), **kw)
        assert "INVAL" in str(ei.value)
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=2)
    sp = wl.systems[0]
    rng = np.random.default_rng(3)
    with pytest.raises(lib.MucaError) as ei:                          # discontinuous ln W
        m.set_weights(0, rng.uniform(0, 1, sp.n_bins), rng.uniform(-1, 1, sp.n_bins),
                      np.zeros(sp.n_bins))
    assert "INVAL" in str(ei.value)
    m.close()


def test_initial_bead_outside_sphere_is_rejected(lib):
    import dataclasses
    wl = dataclasses.replace(workloads.single_chain(), box_kind=workloads.BOX_SPHERE, box_len=5.0)
    with pytest.raises(lib.MucaError) as ei:
        lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=2)
    assert "INVAL" in str(ei.value)


def test_four_walkers_per_wave_limits(lib):
    """Four walkers per wave hold at most 64 beads (four slots of 16 lanes) and need a multiple
    of four walkers per system."""
    wl = workloads.cross_seeding(walkers=4)                       # 76 beads
    with pytest.raises(lib.MucaError) as ei:
        lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers_per_wave=4)
    assert "INVAL" in str(ei.value)
    wl = workloads.single_chain()
    with pytest.raises(lib.MucaError) as ei:
        lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=6, walkers_per_wave=4)
    assert "INVAL" in str(ei.value)


@pytest.mark.parametrize("bounds", [(0.0, 0.0), (0.0, 2.0)])
def test_weight_update_matches_oracle(lib, orc, bounds):
    """Berg's recursion on the device against the oracle, unbounded and with the slopes kept in
    an inverse-temperature range (bounds (0, 2) clip the steep first-iteration tails)."""
    wl = workloads.single_chain()
    b_lo, b_hi = bounds
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=4, precision=0,
                               beta_min=b_lo, beta_max=b_hi)
    W = orc.Weights(wl.systems[0].e_lo, wl.bin_width, wl.systems[0].n_bins, beta_min=b_lo,
                    beta_max=b_hi)
    for it in range(3):
        m.sweep(2000)
        H = m.histogram(0)
        st = m.update_weights()[0]
        W.berg_update(H)
        b, a, g = m.weights(0)
        assert np.array_equal(m.histogram(0, last=True), H)
        assert not m.histogram(0).any()
        assert np.allclose(b, W.beta, rtol=1e-13, atol=1e-12)
        assert np.allclose(g, W.g, rtol=1e-14, atol=0)
        assert np.allclose(a, W.alpha, rtol=1e-12, atol=1e-9)
        cv, pk, lo, hi = orc.flatness(H)
        assert st["iteration"] == it and st["moves"] == int(H.sum())
        assert (st["k_min"], st["k_max"]) == (lo, hi)
        assert st["cvar"] == pytest.approx(cv, rel=1e-12) and st["max_peak"] == pytest.approx(pk, rel=1e-12)
        if b_hi > b_lo:
            assert b.min() >= b_lo and b.max() <= b_hi
        # the oracle continues from the GPU's weights so the next histogram is comparable
        W = orc.Weights(W.e_lo, W.bin_width, W.n_bins, b, a, g, b_lo, b_hi)
    m.close()


@pytest.mark.parametrize("make", [lambda: workloads.batched_chains(n_seq=4, walkers=32),
                                  lambda: workloads.aggregation(walkers=16),
                                  lambda: workloads.cross_seeding(walkers=16)])
def test_fp32_split_resync_restores_fp64_energy(lib, orc, make):
    """FP32 pair terms make the running energy drift between resyncs (bounded by drift_tol);
    right after a resync it equals the FP64 energy of the walker's own coordinates."""
    wl = make()
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), precision=1,
                               resync_sweeps=100, drift_tol=1e-3)
    m.sweep(400)                                         # ends on a resync
    for s in range(wl.n_systems):
        sysd = orc.System.from_workload(wl, s)
        pos, e, cnt = m.walkers_state(s)
        for i in range(pos.shape[0]):
            e64, _, scale = sysd.energy_parts(pos[i])
            assert abs(e[i] - e64) <= 1e-11 * max(1.0, scale), (s, i, e[i], e64, scale)
        assert np.all(cnt["max_drift"] > 0) and np.all(cnt["max_drift"] < 1e-3)
        assert np.all(cnt["accepted"] > 0.05 * cnt["moves"])
        bl = np.linalg.norm(np.diff(pos, axis=1), axis=2)
        starts = np.cumsum([0] + wl.systems[s].chain_len)[:-1]
        keep = np.ones(bl.shape[1], bool)
        keep[starts[1:] - 1] = False                     # skip links between chains
        assert np.max(np.abs(bl[:, keep] - 1.0)) < 1e-12
    m.close()


def test_fp32_resync_drift_and_iterate_graph(lib, orc):
    wl = workloads.aggregation(walkers=64)
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), precision=1,
                               resync_sweeps=50, drift_tol=1e-3)
    m.iterate(200, 3)
    hist = m.stats_history(0, 3)
    assert np.all(hist[:, 0, 0] == 64 * 200 * (36 + 1))        # every trial move counted
    pos, e, cnt = m.walkers_state(0)
    assert np.all(cnt["sweeps"] == 600) and np.all(cnt["max_drift"] < 1e-4)
    m.close()


def test_window_error_is_reported(lib):
    wl = workloads.single_chain()
    sp = wl.systems[0]
    sp.e_lo = 10.0                                       # window above the starting energy
    with pytest.raises(lib.MucaError) as ei:
        lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=1)
    assert "WINDOW" in str(ei.value)


def test_checkpoint_resume_is_bit_identical(lib):
    """Stopping after n sweeps, saving the state and resuming in a fresh context gives exactly
    the trajectory, histogram and weights of an uninterrupted run (counter-based streams carry no
    generator state)."""
    wl = workloads.aggregation(walkers=8)
    p0 = workloads.initial_positions(wl)
    a = lib.Muca.from_workload(wl, p0, precision=1, resync_sweeps=50)
    a.sweep(150)
    a.update_weights()
    a.sweep(100)
    pa, ea, ca = a.walkers_state(0)
    ha = a.histogram(0)
    wa = a.weights(0)
    b = lib.Muca.from_workload(wl, p0, precision=1, resync_sweeps=50)
    b.sweep(150)
    b.update_weights()
    blob = b.get_state()
    b.close()
    c = lib.Muca.from_workload(wl, p0, precision=1, resync_sweeps=50)
    c.set_state(blob)
    c.sweep(100)
    pc, ec, cc = c.walkers_state(0)
    assert np.array_equal(pa, pc) and np.array_equal(ea, ec)
    assert np.array_equal(ha, c.histogram(0))
    for x, y in zip(wa, c.weights(0)):
        assert np.array_equal(x, y)
    for k in ca:
        assert np.array_equal(ca[k], cc[k])
    a.close()
    c.close()


def test_fp64_resume_across_launch_plans(lib):
    """FP64 trajectories do not depend on the launch plan: a run in the mixed plan (16-, 32- and
    64-lane walkers) saved after a weight update and resumed with two walkers per wave ends in
    exactly the state of an uninterrupted run in one walker per wave."""
    wl = workloads.chains_of_lengths([12, 24, 40, 56])
    p0 = workloads.initial_positions(wl)
    a = lib.Muca.from_workload(wl, p0, walkers=4, precision=0, walkers_per_wave=1)
    a.sweep(120)
    a.update_weights()
    a.sweep(80)
    b = lib.Muca.from_workload(wl, p0, walkers=4, precision=0, walkers_per_wave=-1)
    assert b.launch_info()["lanes_used"] == 0b111
    b.sweep(120)
    b.update_weights()
    blob = b.get_state()
    b.close()
    c = lib.Muca.from_workload(wl, p0, walkers=4, precision=0, walkers_per_wave=2)
    c.set_state(blob)
    c.sweep(80)
    for s in range(wl.n_systems):
        pa, ea, ca = a.walkers_state(s)
        pc, ec, cc = c.walkers_state(s)
        assert np.allclose(pa, pc, rtol=0, atol=1e-10)
        assert np.allclose(ea, ec, rtol=0, atol=1e-9)
        assert np.array_equal(a.histogram(s), c.histogram(s))
        for k in ("moves", "accepted", "window_rejects", "sweeps"):
            assert np.array_equal(ca[k], cc[k])
        for x, y in zip(a.weights(s), c.weights(s)):
            assert np.allclose(x, y, rtol=0, atol=1e-12)
    a.close()
    c.close()


def test_drift_detector_fires_on_corrupted_energy(lib):
    """The FP64 resync compares the running energy with a full recomputation and reports
    MUCA_E_DRIFT when they differ by more than drift_tol (here a corrupted running energy)."""
    import struct
    wl = workloads.aggregation(walkers=4)
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), precision=1,
                               resync_sweeps=10, drift_tol=1e-3)
    m.sweep(10)
    blob = bytearray(m.get_state())
    hdr = struct.unpack_from("6Q", blob, 0)
    e_off = 48 + 8 * hdr[2]                               # header, then coordinates
    e0 = struct.unpack_from("d", blob, e_off)[0]
    struct.pack_into("d", blob, e_off, e0 + 0.01)         # walker 0's running energy is off
    m.set_state(bytes(blob))
    m.sweep(10)
    with pytest.raises(lib.MucaError) as ei:
        m.synchronize()
    assert "DRIFT" in str(ei.value)
    m.close()


@pytest.mark.parametrize("pack", [1, 2, 4])
def test_window_edge_tolerance(lib, pack):
    """A running energy up to 1e-3 outside the window (what FP32 accumulation can leave at an edge
    until the next FP64 resync) is kept in the edge bin; further outside it is an error."""
    import struct
    wl = workloads.single_chain()
    sp = wl.systems[0]
    e_hi = sp.e_lo + sp.n_bins * wl.bin_width
    for offset, ok in ((5e-4, True), (1e-2, False)):
        m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=4, precision=1,
                                   resync_sweeps=10, walkers_per_wave=pack)
        blob = bytearray(m.get_state())
        hdr = struct.unpack_from("6Q", blob, 0)
        struct.pack_into("d", blob, 48 + 8 * hdr[2], e_hi + offset)
        m.set_state(bytes(blob))
        m.sweep(20)
        if ok:
            m.synchronize()
            _, e, _ = m.walkers_state(0)
            assert np.all(e < e_hi)                    # resync restored the exact energy
        else:
            with pytest.raises(lib.MucaError) as ei:
                m.synchronize()
            assert "WINDOW" in str(ei.value)
        m.close()


@pytest.mark.parametrize("side", ["top", "bottom"])
@pytest.mark.parametrize("pack", [1, 2])
def test_fp64_running_energy_just_outside_the_window_matches_oracle(lib, orc, side, pack):
    """The window-edge rule against the reference's edge reading (edge_tol = 1e-3), move for
    move in FP64: every walker's running energy is set 5e-4 outside the window, as FP32
    accumulation can leave it at an edge until the next resync.  Both sides continue from the edge
    bin with that energy (ln W extends the bin's line), count their moves there until a move
    enters the window, and must agree in accept sequences, histograms and coordinates."""
    import struct
    wl = workloads.single_chain()
    sp = wl.systems[0]
    s = orc.System.from_workload(wl)
    K = sp.n_bins
    beta = np.full(K, 1 / 0.7)
    # a random coil (from the straight start nearly every move raises the energy)
    Wc = orc.Weights(sp.e_lo, wl.bin_width, K, beta, np.zeros(K))
    wc = orc.Walker(s, workloads.initial_positions(wl)[0], 7, wl.seed)
    wc.run(Wc, orc.move_params(wl), 200, np.zeros(K, np.uint64))
    coil = wc.pos.copy()
    top = sp.e_lo + K * wl.bin_width
    e_start = top + 5e-4 if side == "top" else sp.e_lo - 5e-4
    n_walk, n_sweeps = 4, 60
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=n_walk, precision=0,
                               walkers_per_wave=pack)
    m.set_weights(0, beta, np.zeros(K), np.zeros(K))
    m.set_walkers(0, np.repeat(coil[None], n_walk, axis=0))
    blob = bytearray(m.get_state())
    n_pos = struct.unpack_from("6Q", blob, 0)[2]
    for i in range(n_walk):
        struct.pack_into("d", blob, 48 + 8 * n_pos + 8 * i, e_start)
    m.set_state(bytes(blob))
    n_log = n_sweeps * sp.n_beads
    m.set_accept_log(n_log)
    m.sweep(n_sweeps)
    W = orc.Weights(sp.e_lo, wl.bin_width, K, beta, np.zeros(K), edge_tol=1e-3)
    H = np.zeros(K, np.uint64)
    log_g = m.accept_log(0)
    pos_g, e_g, cnt = m.walkers_state(0)
    edge = K - 1 if side == "top" else 0
    for i in range(n_walk):
        ow = orc.Walker(s, coil, i, wl.seed)
        ow.energy = e_start
        log = np.zeros(n_log, np.uint8)
        h_before = int(H[edge])
        ow.run(W, orc.move_params(wl), n_sweeps, H, accept_log=log)
        assert int(H[edge]) > h_before, "no move counted in the edge bin"
        assert np.array_equal(log_g[i], log), f"accept sequence of walker {i} differs"
        assert np.allclose(pos_g[i], ow.pos, rtol=0, atol=1e-10)
        assert e_g[i] == pytest.approx(ow.energy, abs=1e-9)
        assert cnt["window_rejects"][i] == ow.counters.window_rejects
    assert np.array_equal(m.histogram(0), H)
    m.close()


def test_discontinuous_weights_fall_back_to_one_walker_per_wave(lib, orc):
    """Two walkers per wave read ln W from its bin-edge values, which needs continuous weights.
    Random (discontinuous) beta, alpha switch the context to one walker per wave, whose sweep still
    matches the oracle move for move; continuous weights switch it back."""
    wl = workloads.single_chain()
    sp = wl.systems[0]
    rng = np.random.default_rng(5)
    beta = rng.uniform(0.0, 0.5, sp.n_bins)
    alpha = rng.uniform(-2.0, 2.0, sp.n_bins)
    g = np.zeros(sp.n_bins)
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=4, precision=0)
    assert m.launch_info()["walkers_per_wave"] == 2
    m.set_weights(0, beta, alpha, g)
    assert m.launch_info()["walkers_per_wave"] == 1
    n_sweeps = 500
    m.set_accept_log(n_sweeps * sp.n_beads)
    m.sweep(n_sweeps)
    W = orc.Weights(sp.e_lo, wl.bin_width, sp.n_bins, beta, alpha, g)
    H, ows = _oracle_walkers(orc, wl, 0, 4, n_sweeps, W, log_moves=n_sweeps * sp.n_beads)
    assert np.array_equal(m.histogram(0), H)
    log_g = m.accept_log(0)
    pos_g, e_g, _ = m.walkers_state(0)
    for i, (ow, olog) in enumerate(ows):
        assert np.array_equal(log_g[i], olog)
        assert np.allclose(pos_g[i], ow.pos, rtol=0, atol=1e-10)
    res = orc.muca(wl, n_iter=2, n_sweeps=2000, walkers=2)
    Wc = res["weights"]
    m.set_weights(0, Wc.beta, Wc.alpha, Wc.g)
    assert m.launch_info()["walkers_per_wave"] == 2
    m.close()


@pytest.mark.parametrize("pack", [1, 2])
def test_fp64_largest_system(lib, orc, pack):
    """128 beads, the largest system a context holds (two bead slots of 64 lanes, or four of 32),
    with a 2000-bin window around the starting energy."""
    wl = workloads.single_chain(n=128)
    sp = wl.systems[0]
    sp.e_lo, sp.n_bins = -40.0, 2000
    _compare(lib, orc, wl, walkers=2, n_sweeps=60, pack=pack)


@pytest.mark.parametrize("pack", [1, 2, 4])
def test_fp64_shortest_chain(lib, orc, pack):
    """Three beads: one interior bead, two ends, a single non-bonded pair."""
    wl = workloads.single_chain(n=3)
    _compare(lib, orc, wl, walkers=_walkers(pack, 2), n_sweeps=1000, pack=pack)


def test_zero_sweeps_is_a_no_op(lib):
    wl = workloads.single_chain()
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=2)
    p0, e0, c0 = m.walkers_state(0)
    m.sweep(0)
    p1, e1, c1 = m.walkers_state(0)
    assert np.array_equal(p0, p1) and np.array_equal(e0, e1)
    assert not m.histogram(0).any() and np.all(c1["moves"] == 0)
    m.close()
