"""GPU hybrid Monte Carlo (muca_hmc) against the FP64 reference oracle/hmc.py through the C ABI:
same Philox momenta and acceptance draws, so every walker must take the same decisions, end at
the same coordinates (to rounding) and fill the same histogram, on a single chain, the periodic
aggregation workload and the steric sphere; plus the entry point's limits and checkpointing."""
import dataclasses

import numpy as np
import pytest

import workloads
from oracle import hmc as HM

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1702_01770_amd as P
    P.load()
    return P


def _canonical(sp, wl, T):
    return np.full(sp.n_bins, 1.0 / T), np.zeros(sp.n_bins), np.zeros(sp.n_bins)


@pytest.mark.parametrize("make,T,steps,h", [
    (lambda: workloads.single_chain(), 0.6, 8, 0.05),
    (lambda: workloads.aggregation(walkers=4), 0.8, 6, 0.04),
    (lambda: workloads.confined(radius=6.0, walkers=4), 0.8, 6, 0.05),
    (lambda: workloads.paper_system("abeta_dimer", walkers=4), 0.7, 6, 0.05),
    # the largest chain one wave holds: every lane a bead, partners wrap at lane 63, and the
    # pairs at offset N/2 = 32 are taken by the lower half of the lanes only
    (lambda: workloads.single_chain(n=64), 0.6, 8, 0.03),
])
def test_hmc_matches_oracle(lib, orc, make, T, steps, h):
    wl = make()
    sp = wl.systems[0]
    n_walk, n_traj = 4, 25
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=n_walk, precision=0)
    b, a, g = _canonical(sp, wl, T)
    m.set_weights(0, b, a, g)
    m.hmc(n_traj, steps, h)
    Hg = m.histogram(0)
    pos_g, e_g, cnt = m.walkers_state(0)
    W = orc.Weights(sp.e_lo, wl.bin_width, sp.n_bins, b, a)
    s = orc.System.from_workload(wl)
    sphere_r2 = wl.box_len ** 2 if wl.box_kind == workloads.BOX_SPHERE else 0.0
    H = np.zeros(sp.n_bins, np.uint64)
    total_acc = 0
    for i in range(n_walk):
        w = HM.HmcWalker(s, workloads.initial_positions(wl)[0], i, wl.seed)
        rec = []
        for _ in range(n_traj):
            w.trajectory(W, steps, h, H, sphere_r2, record=rec)
        _, _, scale = s.energy_parts(w.pos)
        assert cnt["hmc_trajectories"][i] == n_traj
        assert cnt["hmc_accepted"][i] == w.accepted, (i, cnt["hmc_accepted"][i], w.accepted)
        # A trajectory that ends outside the window is rejected for that reason (R28).  One whose
        # Hamiltonian blows up (overlapping beads: H1 - H0 > 30, acceptance below e^-30) ends in a
        # state that rounding decides chaotically, inside or outside the window; both sides reject
        # it, but which rule fires may differ.  Every other trajectory must agree on the reason.
        chaotic = sum(1 for r in rec if not r["accept"] and not (r["H1"] - r["H0"] <= 30.0))
        assert abs(int(cnt["window_rejects"][i]) - w.window_rejects) <= chaotic, (
            i, cnt["window_rejects"][i], w.window_rejects, chaotic)
        # the momenta's transcendentals differ from glibc's in the last ulp and the dynamics
        # amplify that: positions agree to 1e-8, the energy is exact for the GPU's own positions
        assert np.allclose(pos_g[i], w.pos, rtol=0, atol=1e-8), (i, np.abs(pos_g[i] - w.pos).max())
        _, _, own_scale = s.energy_parts(pos_g[i])
        assert abs(e_g[i] - s.energy(pos_g[i])) <= 1e-11 * max(1.0, own_scale)
        assert abs(e_g[i] - w.energy) <= 1e-7 * max(1.0, scale)
        bl = np.linalg.norm(np.diff(pos_g[i], axis=0), axis=1)
        ends = np.cumsum(sp.chain_len)[:-1] - 1
        assert np.max(np.abs(np.delete(bl, ends) - 1.0)) < 1e-12
        total_acc += w.accepted
    assert np.array_equal(Hg, H)
    assert 0 < total_acc < n_walk * n_traj            # a real test: some accepted, some not
    m.close()


def test_hmc_then_sweeps_continue_from_the_same_state(lib, orc):
    """Hybrid MC and single-bead sweeps share the walkers: after the trajectories the running
    energy is the FP64 energy of the coordinates, and the following sweeps (coordinates reloaded
    into LDS, the walker's sweep counter untouched by HMC) match, move for move, an oracle walker
    continued from the GPU's coordinates with the same walker id and stream position."""
    wl = workloads.single_chain()
    sp = wl.systems[0]
    n_walk, n_sweeps = 4, 400
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=n_walk, precision=0)
    b, a, g = _canonical(sp, wl, 0.7)
    m.set_weights(0, b, a, g)
    m.hmc(10, 6, 0.05)
    pos_h, e_h, cnt_h = m.walkers_state(0)
    s = orc.System.from_workload(wl)
    for i in range(n_walk):
        assert abs(e_h[i] - s.energy(pos_h[i])) < 1e-10 * max(1.0, s.energy_parts(pos_h[i])[2])
    assert np.all(cnt_h["sweeps"] == 0) and np.all(cnt_h["hmc_trajectories"] == 10)
    assert 0 < cnt_h["hmc_accepted"].sum() < 10 * n_walk
    H_after_hmc = m.histogram(0).copy()
    n_log = n_sweeps * sp.n_beads
    m.set_accept_log(n_log)
    m.sweep(n_sweeps)
    log_g = m.accept_log(0)
    pos_g, e_g, cnt = m.walkers_state(0)
    H_sweep = m.histogram(0) - H_after_hmc
    W = orc.Weights(sp.e_lo, wl.bin_width, sp.n_bins, b, a, g)
    H = np.zeros(sp.n_bins, np.uint64)
    for i in range(n_walk):
        ow = orc.Walker(s, pos_h[i], i, wl.seed)
        assert ow.energy == pytest.approx(e_h[i], abs=1e-11)
        log = np.zeros(n_log, np.uint8)
        ow.run(W, orc.move_params(wl), n_sweeps, H, accept_log=log)
        assert np.array_equal(log_g[i], log), f"walker {i}: accept sequence after HMC differs"
        assert np.allclose(pos_g[i], ow.pos, rtol=0, atol=1e-10)
        assert e_g[i] == pytest.approx(ow.energy, abs=1e-10)
        assert cnt["accepted"][i] == ow.counters.accepted
        assert cnt["sweeps"][i] == n_sweeps
    assert np.array_equal(H_sweep, H)
    m.close()


def test_hmc_after_fp32_split_sweeps_starts_from_the_fp64_energy(lib, orc):
    """In the FP32-split mode the running energy of the sweeps drifts from the FP64 energy of the
    coordinates (no resync here).  The trajectories build H0 from the FP64 energy of the start,
    so their decisions are those of an FP64 oracle walker started from the GPU's coordinates,
    and afterwards the walker's energy is exact again (a rejected trajectory keeps the
    recomputed start energy)."""
    wl = workloads.batched_chains(n_seq=1, n_min=40, n_max=40)
    sp = wl.systems[0]
    n_walk, n_traj, steps, h = 4, 20, 6, 0.03
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=n_walk, precision=1,
                               resync_sweeps=0)
    b, a, g = _canonical(sp, wl, 0.7)
    m.set_weights(0, b, a, g)
    m.sweep(3000)
    pos0, e0, _ = m.walkers_state(0)
    s = orc.System.from_workload(wl)
    drift = np.array([abs(e0[i] - s.energy(pos0[i])) for i in range(n_walk)])
    print("running-energy drift before HMC", drift)
    assert drift.max() > 1e-9, "no drift to test against"
    H0 = m.histogram(0).copy()
    m.hmc(n_traj, steps, h)
    pos_g, e_g, cnt = m.walkers_state(0)
    W = orc.Weights(sp.e_lo, wl.bin_width, sp.n_bins, b, a)
    H = np.zeros(sp.n_bins, np.uint64)
    for i in range(n_walk):
        w = HM.HmcWalker(s, pos0[i], i, wl.seed)
        for _ in range(n_traj):
            w.trajectory(W, steps, h, H)
        assert cnt["hmc_accepted"][i] == w.accepted, (i, cnt["hmc_accepted"][i], w.accepted)
        assert np.allclose(pos_g[i], w.pos, rtol=0, atol=1e-8)
        _, _, sc = s.energy_parts(pos_g[i])
        assert abs(e_g[i] - s.energy(pos_g[i])) <= 1e-11 * max(1.0, sc)
    assert np.array_equal(m.histogram(0) - H0, H)
    m.close()


def test_hmc_limits_and_checkpoint(lib):
    wl = workloads.cross_seeding()                     # 76 beads: more than one wave holds
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=2)
    with pytest.raises(lib.MucaError):
        m.hmc(1, 4, 0.05)
    m.close()
    wl = workloads.single_chain()
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=2, precision=0)
    for bad in ((1, 0, 0.05), (1, 4, 0.0), (-1, 4, 0.05)):
        with pytest.raises(lib.MucaError):
            m.hmc(*bad)
    m.hmc(3, 5, 0.05)
    st = m.get_state()
    m.hmc(4, 5, 0.05)
    p1, e1, c1 = m.walkers_state(0)
    m.set_state(st)
    m.hmc(4, 5, 0.05)
    p2, e2, c2 = m.walkers_state(0)
    assert np.array_equal(p1, p2) and np.array_equal(e1, e2)
    assert np.array_equal(c1["hmc_trajectories"], c2["hmc_trajectories"])
    assert np.all(c1["hmc_trajectories"] == 7)
    m.close()
