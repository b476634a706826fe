"""Parity at the benchmark's full sizes and launch configurations, on sampled outputs the oracle
computes one by one: the batched workload (32 systems, 4096 walkers; two walkers per wave in
paired workgroups, the mixed plan, and the plan the autotuner picks for the benchmark) in FP64
mode against oracle walkers of the same index, the same workload in the benchmarked FP32-split
mode against the FP64 energy of each sampled walker's coordinates, and the energy kernels on
10^6 configurations."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

SAMPLED_SYSTEMS = (0, 7, 19, 31)
SAMPLED_WALKERS = (0, 1, 63, 126, 127)       # walker index within its system


@pytest.fixture(scope="module")
def lib():
    import paper_1702_01770_amd as P
    P.load()
    return P


@pytest.mark.parametrize("plan", ["two_per_wave", "mixed", "autotuned"])
def test_batched_full_size_fp64_sampled_walkers(lib, orc, plan):
    """FP64 trajectories of sampled walkers in the two-walkers-per-wave plan, the mixed plan
    with every qualifying system on whole waves, and whatever plan the autotuner picks (the
    benchmark's)."""
    wl = workloads.batched_chains()
    n_sweeps = 12
    kw = dict(walkers_per_wave=2, waves_per_block=8) if plan == "two_per_wave" else (
        dict(walkers_per_wave=-1) if plan == "mixed" else {})
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), precision=0, **kw)
    if plan == "autotuned":
        m.autotune(probe_sweeps=20)
    info = m.launch_info()
    print("launch plan", info)
    assert info["workgroups"] <= 256
    if plan == "two_per_wave":
        assert info["walkers_per_wave"] == 2 and info["paired"] == 1 and info["workgroups"] == 256
    if plan == "mixed":
        assert info["walkers_per_wave"] == -1 and info["lanes_used"] == 0b111
    n_log = n_sweeps * min(sp.n_beads for sp in wl.systems)
    m.set_accept_log(n_log)
    m.sweep(n_sweeps)
    mv = orc.move_params(wl)
    for s in SAMPLED_SYSTEMS:
        sp = wl.systems[s]
        osys = orc.System.from_workload(wl, s)
        pos_g, e_g, cnt = m.walkers_state(s)
        log_g = m.accept_log(s)
        for i in SAMPLED_WALKERS:
            w = orc.Walker(osys, workloads.initial_positions(wl)[s], s * wl.walkers_per_system + i,
                           wl.seed)
            H = np.zeros(sp.n_bins, np.uint64)
            log = np.zeros(n_log, np.uint8)
            w.run(orc.Weights(sp.e_lo, wl.bin_width, sp.n_bins), mv, n_sweeps, H, accept_log=log)
            assert np.array_equal(log_g[i], log), (s, i)
            _, _, scale = osys.energy_parts(w.pos)
            assert np.allclose(pos_g[i], w.pos, rtol=0, atol=1e-10), (s, i)
            assert abs(e_g[i] - w.energy) <= 1e-11 * max(1.0, scale), (s, i)
            assert cnt["accepted"][i] == w.counters.accepted
    m.close()


@pytest.mark.parametrize("plan", ["two_per_wave", "autotuned"])
def test_batched_full_size_fp32_split_energies(lib, orc, plan):
    """The benchmarked mode (FP32 pair terms, FP64 resync every 100 sweeps) after two MUCA
    iterations, in the two-walkers plan and in the autotuned plan the benchmark runs: every
    sampled walker's running energy is the FP64 energy of its coordinates within 1e-5 of the sum
    of term magnitudes, its bonds are unit, and every trial move was counted once in its
    system's histogram."""
    wl = workloads.batched_chains()
    n_sweeps = 250
    kw = dict(walkers_per_wave=2, waves_per_block=8) if plan == "two_per_wave" else {}
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), **kw)
    if plan == "autotuned":
        m.autotune(probe_sweeps=500)
        print("launch plan", m.launch_info())
    m.iterate(n_sweeps, 2)
    st = m.stats_history(0, 2)
    for s in SAMPLED_SYSTEMS:
        sp = wl.systems[s]
        assert st[1, s, 0] == wl.walkers_per_system * n_sweeps * sp.n_beads
        osys = orc.System.from_workload(wl, s)
        pos_g, e_g, _ = m.walkers_state(s)
        for i in SAMPLED_WALKERS:
            e64 = osys.energy(pos_g[i])
            _, _, scale = osys.energy_parts(pos_g[i])
            assert abs(e_g[i] - e64) <= 1e-5 * scale, (s, i, e_g[i], e64)
            bl = np.linalg.norm(np.diff(pos_g[i], axis=0), axis=1)
            assert np.max(np.abs(bl - 1.0)) < 1e-9
    m.close()


def test_energy_kernels_on_a_million_configurations(lib, orc):
    """10^6 configurations (2000 distinct cross-seeding geometries tiled 500 times) in the
    differentiation leg's launch configuration: sampled energies and gradients against the
    oracle, and every copy of a geometry bit-identical to its first copy."""
    import torch
    wl = workloads.cross_seeding()
    sp = wl.systems[0]
    base = workloads.random_bond_chains(41, 2000, sp.chain_len, box_len=wl.box_len)
    x32 = base.astype(np.float32)
    reps = 500
    xt = torch.tensor(x32, device="cuda").repeat(reps, 1, 1).contiguous()
    assert xt.shape[0] == 1_000_000
    theta = np.array([wl.c_lj[0, 1], wl.c_lj[1, 1], wl.k_bend, wl.k_tors])
    m = lib.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=2)
    E = torch.empty(xt.shape[0], dtype=torch.float64, device="cuda")
    m.energy_fwd_ptr(0, xt.data_ptr(), xt.shape[0], theta, E.data_ptr())
    ge = torch.ones_like(E)
    gx = torch.empty_like(xt)
    gth = torch.empty(4, dtype=torch.float64, device="cuda")
    m.energy_bwd_ptr(0, xt.data_ptr(), xt.shape[0], theta, ge.data_ptr(), gx.data_ptr(),
                     gth.data_ptr())
    m.synchronize()
    Eh = E.cpu().numpy().reshape(reps, -1)
    gxh = gx.cpu().numpy().reshape(reps, 2000, sp.n_beads, 3)
    assert np.array_equal(Eh, np.broadcast_to(Eh[0], Eh.shape))
    assert np.array_equal(gxh, np.broadcast_to(gxh[0], gxh.shape))
    s = orc.System.from_workload(wl)
    gth_ref = np.zeros(4)
    for i in range(2000):
        e64, grad, dth = s.energy_grad(x32[i].astype(np.float64))
        gth_ref += dth
        if i % 97 == 0:
            _, _, scale = s.energy_parts(x32[i].astype(np.float64))
            assert abs(Eh[0, i] - e64) <= 1e-5 * scale
            assert np.max(np.abs(gxh[0, i] - grad)) <= 2e-4 * (np.abs(grad).max() + 1e-30)
    assert np.allclose(gth.cpu().numpy(), reps * gth_ref, rtol=1e-4,
                       atol=1e-6 * np.abs(reps * gth_ref).max())
    m.close()
