"""Benchmark: multicanonical (MUCA) trial moves per second on one MI355X.

Workload (synthetic stand-in for the paper's chains, see workloads.batched_chains): 32 single-chain
AB systems with lengths drawn uniformly from 13..55 (~60 % A), 128 walkers per system (4096
walkers), bin width 0.05 over [-4N, +N), FP32 pair arithmetic with FP64 energies / weights.
One step = one MUCA iteration: --sweeps sweeps of every walker followed by the Berg weight
update, replayed from a captured HIP graph (persistent sweep launches + update kernel).

Printed JSON line: value = single-bead trial moves per second over all walkers (batched form),
plus the plain form (one walker per system, same kernels) for comparison, the roofline of the
sweep kernel (algorithmic FP32/FP64 ALU operations per launch over the launch time measured
with HIP events on the library's stream) and the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X vector FP32 (published, packed)


def algorithmic_flops_per_move(n_beads: int, n_chains: int = 1, periodic: bool = False,
                               torsion: bool = False) -> float:
    """Operations a single-bead trial move must perform (no Newton refinements, no masked
    work): per non-bonded partner two pair-term evaluations (separation 3, r^2 5, reciprocal 1,
    s^3 2, s^3 (kappa s^3 - kappa C) 2 = 13 each; +9 each for the periodic minimum image) plus
    their difference and the accumulation (2); 50 for the bending terms, +56 with torsion; 60 for
    building the proposal and the acceptance test."""
    bonded = (2 * (n_beads - 2 * n_chains) + 2 * n_chains) / n_beads   # mean bonded neighbours
    partners = n_beads - 1 - bonded
    per_pair = 2 * (13 + (9 if periodic else 0)) + 2
    return partners * per_pair + 50 + 60 + (56 if torsion else 0)


_STREAMS = []


def make_stream():
    """A non-default torch stream for the library (kept alive for the whole run)."""
    import torch
    torch.cuda.set_device(0)
    s = torch.cuda.Stream()
    _STREAMS.append(s)
    return s


def run_gpu(wl, walkers, n_sweeps, steps, warmup, stream, autotune=True, **launch):
    """Run `warmup` then `steps` MUCA iterations; time the steps with HIP events recorded on the
    stream the library launches on."""
    import torch

    import paper_1702_01770_amd as P
    import workloads
    m = P.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=walkers,
                             stream=stream.cuda_stream, **launch)
    # probes of a fixed length, so that the plan does not depend on the sweeps per iteration
    chosen = m.autotune(probe_sweeps=min(500, max(5, n_sweeps))) if autotune else None
    plan = m.launch_info()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    if warmup:
        m.iterate(n_sweeps, warmup)
    m.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    m.iterate(n_sweeps, steps)
    e1.record(stream)
    m.synchronize()
    e1.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    stats = m.stats_history(warmup, steps)
    moves = 0
    for s, sp in enumerate(wl.systems):
        moves += walkers * n_sweeps * sp.n_beads * steps
    _, _, cnt = m.walkers_state(0)
    m.close()
    launches = steps * -(-n_sweeps // plan["sweeps_per_launch"])
    return dict(moves=moves, event_ms=ms, wall_s=wall, stats=stats, chosen=chosen, plan=plan,
                launches=launches,
                acc_rate=float(np.sum(cnt["accepted"]) / max(1, np.sum(cnt["moves"]))))


def matched_error(stream):
    """Batched vs plain at the same statistics per MUCA iteration, on the 6-bead chain whose
    FP64-oracle replica statistics are stored in tests/golden/muca_n6_reference.json.  Plain: one
    walker doing all sweeps of an iteration; batched: 64 walkers sharing the weights, each doing
    1/64 of them.  Reports the S(E) error of each against the oracle replica mean (RMS over the
    grid, in units of the oracle's replica standard deviation) and the GPU time of each run."""
    import torch

    import paper_1702_01770_amd as P
    import workloads
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "muca_n6_reference.json")))
    oS = np.array([c["S"] for c in ref["curves"]])
    o_mean, o_sd = oS.mean(axis=0), oS.std(axis=0, ddof=1)
    total = ref["walkers"] * ref["sweeps"]
    iters, block, k_lo, k_hi = ref["iterations"], ref["block"], ref["k_lo"], ref["k_hi"]
    out = {}
    for name, walkers in (("plain", 1), ("batched", 64)):
        wl = workloads.single_chain(n=6)
        sp = wl.systems[0]
        reps = 4
        wl.systems = [sp] * reps                       # 4 independent replicas at once
        m = P.Muca.from_workload(wl, workloads.initial_positions(workloads.single_chain(n=6)) * reps,
                                 walkers=walkers, precision=1, seed=77_000_003,
                                 resync_sweeps=100, stream=stream.cuda_stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        bs = [[] for _ in range(reps)]
        al = [[] for _ in range(reps)]
        ms_total = 0.0
        for _ in range(iters):
            e0.record(stream)
            m.sweep(total // walkers)
            e1.record(stream)
            m.update_weights()
            e1.synchronize()
            ms_total += e0.elapsed_time(e1)
            for r in range(reps):
                b, a, _ = m.weights(r)
                bs[r].append(b)
                al[r].append(a)
        m.close()
        errs = []
        for r in range(reps):
            res = P.microcanonical_analyze(np.array(bs[r]), np.array(al[r]), sp.e_lo,
                                           wl.bin_width, k_lo, k_hi, iters - block, iters,
                                           block, wl.bin_width, beta_c=1.0)
            d = (res["S"] - o_mean)[:-1] / o_sd[:-1]
            errs.append(float(np.sqrt(np.mean(d * d))))
        out[name] = {"walkers": walkers, "sweeps_per_walker_per_iter": total // walkers,
                     "gpu_ms_per_iter": ms_total / iters,
                     "S_rms_err_in_oracle_sd": float(np.mean(errs))}
    out["time_ratio_plain_over_batched"] = (out["plain"]["gpu_ms_per_iter"] /
                                            out["batched"]["gpu_ms_per_iter"])
    out["system"] = "single chain N=6 (workloads.single_chain(n=6)), 4 replicas per form"
    return out


def chain_moves_leg(wl, stream, sweeps=2000, steps=2):
    """The batched workload with one pivot after every sweep (the paper's pivotings): single-bead
    moves and pivots per second, same kernels and schedule search."""
    import dataclasses
    w2 = dataclasses.replace(wl, pivot_per_sweep=1)
    r = run_gpu(w2, w2.walkers_per_system, sweeps, steps, 1, stream)
    sec = r["event_ms"] / 1e3
    pivots = w2.walkers_per_system * len(w2.systems) * sweeps * steps
    return {"pivot_per_sweep": 1, "sweeps_per_step": sweeps, "steps": steps,
            "single_bead_moves_per_s": r["moves"] / sec, "pivots_per_s": pivots / sec,
            "ms_per_step": r["event_ms"] / steps, "launch_plan": r["plan"]}


def paper_systems_leg(stream, sweeps=2000, steps=2):
    """The A/B strings the paper prints for its examples (Sec. 4.1, 4.2) in its steric spheres,
    4096 walkers each, with one rigid translation, one pivot and one chain rotation after every
    sweep: single-bead trial moves per second (the chain-level moves run on top)."""
    import workloads
    out = {}
    for name in workloads.PAPER_SYSTEMS:
        wl = workloads.paper_system(name)
        r = run_gpu(wl, wl.walkers_per_system, sweeps, steps, 1, stream)
        sec = r["event_ms"] / 1e3
        per_sweep = wl.rigid_per_sweep + wl.pivot_per_sweep + wl.rotate_per_sweep
        chain_moves = per_sweep * wl.walkers_per_system * sweeps * steps
        out[name] = {"beads": wl.systems[0].n_beads, "sphere_radius": wl.box_len,
                     "single_bead_moves_per_s": r["moves"] / sec,
                     "chain_level_moves_per_s": chain_moves / sec,
                     "ms_per_step": r["event_ms"] / steps, "launch_plan": r["plan"]}
    out["sweeps_per_step"] = sweeps
    return out


# Latent heats and free-energy barriers the paper reports for its cross-seeding systems
# (Sec. 4.2, intensive units): context for the physics leg, not a parity target (the paper's
# force-field details and statistics differ).
PAPER_MAXWELL = {"cross_human": {"latent": 0.513, "barrier": 0.034},
                 "cross_rat": {"latent": 0.584, "barrier": 0.021}}


# Sweeps per MUCA iteration, summed over all walkers, in the paper's runs (Sec. 4.1: 10^6 for the
# dimer; Sec. 4.2: 10^7 for the cross-seeding mixtures).
PAPER_SWEEPS_PER_ITERATION = {"abeta_dimer": 10 ** 6, "cross_human": 10 ** 7, "cross_rat": 10 ** 7}


def paper_physics_leg(stream, names, iters=1000, walkers=4096, first=700, block=25,
                      hmc_traj=0, hmc_steps=10, hmc_step=0.01, reset_every=0, e_hi=None):
    """Full multicanonical runs of the paper's example systems as in Sec. 4: `walkers` walkers
    share the paper's sweeps per iteration, `iters` Berg iterations, then the
    microcanonical analysis (Eqs. 4-8) of iterations [first, iters) in blocks of `block`:
    Maxwell construction on beta(eps), latent heat and free-energy barrier per monomer, and
    whether the caloric curve bends back (a region of negative microcanonical specific heat).
    Flatness per iteration as the paper judges it: c_var < 5 % and peaks within 20 %.  With
    hmc_traj > 0 every iteration also runs that many hybrid Monte Carlo trajectories per walker
    (hmc_steps leapfrog steps of hmc_step) before the weight update.  With reset_every > 0 the
    recursion's accumulated statistics g are cleared every reset_every iterations before the
    analysed range, so estimates from the early, far-from-equilibrium iterations stop weighing
    on the weights.  e_hi (total energy) moves the window's upper edge from +N."""
    import paper_1702_01770_amd as P
    import workloads
    out = {}
    for name in names:
        wl = workloads.paper_system(name, walkers=walkers, e_hi=e_hi)
        sp = wl.systems[0]
        sweeps = -(-PAPER_SWEEPS_PER_ITERATION[name] // walkers)
        m = P.Muca.from_workload(wl, workloads.initial_positions(wl),
                                 walkers=wl.walkers_per_system, stream=stream.cuda_stream)
        m.autotune(probe_sweeps=20)
        B = np.zeros((iters, sp.n_bins))
        A = np.zeros((iters, sp.n_bins))
        t0 = time.perf_counter()
        for it in range(iters):
            if hmc_traj > 0:
                m.sweep(sweeps)
                m.hmc(hmc_traj, hmc_steps, hmc_step)
                m.update_weights()
            else:
                m.iterate(sweeps, 1)
            B[it], A[it], g_now = m.weights(0)
            if reset_every > 0 and it < first and (it + 1) % reset_every == 0:
                m.set_weights(0, B[it], A[it], np.zeros_like(g_now))
            if (it + 1) % 50 == 0:
                st = m.stats_history(it, 1)[0, 0]
                print(f"[physics] {name} iteration {it + 1}/{iters} cvar {st[1]:.3f} "
                      f"peak {st[2]:.3f} bins [{int(st[3])}, {int(st[4])}] "
                      f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
        st = m.stats_history(0, iters)[:, 0]
        h_last = m.histogram(0, last=True).astype(np.float64)
        m.close()
        flat = (st[:, 1] < 0.05) & (st[:, 2] < 0.20)
        conv = next((i for i in range(iters) if flat[i:].all()), None)
        lo = int(np.max(st[first:, 3])) + 5
        hi = int(np.min(st[first:, 4])) - 5
        if hi - lo < 20:
            out[name] = {"error": f"visited range [{lo}, {hi}) too narrow to analyse",
                         "flat_iterations": int(flat.sum())}
            continue
        inner = h_last[lo:hi]
        inner_cvar = float(inner.std() / inner.mean()) if inner.mean() > 0 else None
        res = P.microcanonical_analyze(B, A, sp.e_lo, wl.bin_width, lo, hi, first, iters, block,
                                       5 * wl.bin_width, beta_c=0.0, tol_beta=1e-3, tol_l=0.02,
                                       n_monomers=sp.n_beads)
        dbeta = np.diff(res["beta"])
        rec = {"beads": sp.n_beads, "sphere_radius": wl.box_len, "iterations": iters,
               "window": [sp.e_lo, sp.e_lo + sp.n_bins * wl.bin_width],
               "sweeps_per_iteration": sweeps * wl.walkers_per_system,
               "walkers": walkers, "hmc_trajectories_per_iteration": hmc_traj,
               "recursion_reset_every": reset_every,
               "flat_iterations": int(flat.sum()), "flat_from": conv,
               "last_cvar_full_range": float(st[-1, 1]), "last_cvar_analysed_range": inner_cvar,
               "eps_range": [float(res["E"][0]), float(res["E"][-1])],
               "beta_c": res["beta_c"], "dbeta_c": res["dbeta_c"],
               "latent_heat": res["latent"], "dlatent_heat": res["dlatent"],
               "barrier": res["barrier"], "dbarrier": res["dbarrier"],
               "backbending": bool(np.any(dbeta > 0)),
               "negative_cv_points": int(np.sum(res["cv"] < 0)),
               "wall_s": time.perf_counter() - t0}
        if name in PAPER_MAXWELL:
            rec["paper"] = PAPER_MAXWELL[name]
        out[name] = rec
    return out


def hmc_flops_per_step(chain_len, periodic=False):
    """Operations one leapfrog step of one walker must perform: every unordered non-bonded pair
    once (separation 3, +9 periodic, r^2 5, reciprocal 1, s^3 2, pair energy 3, force scalar 4,
    force vector 3, added to both beads 6), every bending / torsion term once (value and bond
    derivatives 49, scattered to its beads 9), and per bead the two half kicks with the tangent
    projection (2 x 9), the drift (great-circle turn with cosine and sine, renormalisation and
    projection: 30) and the position and force scans (2 x 3 x 6)."""
    n = int(np.sum(chain_len))
    m = len(chain_len)
    pairs = n * (n - 1) // 2 - (n - m)
    angles = sum(max(0, L - 2) for L in chain_len) + sum(max(0, L - 3) for L in chain_len)
    return pairs * (27 + (9 if periodic else 0)) + angles * 58 + n * (18 + 30 + 36)


def hmc_leg(stream, n_traj=10, n_steps=10, step=0.01):
    """Hybrid Monte Carlo on the batched workload (4096 walkers, 32 single chains of 13..55
    beads) under the weights of one 2000-sweep MUCA iteration: trajectories, leapfrog steps and
    algorithmic FP64 operations per second, timed with HIP events on the library's stream."""
    import torch

    import paper_1702_01770_amd as P
    import workloads
    wl = workloads.batched_chains()
    m = P.Muca.from_workload(wl, workloads.initial_positions(wl), stream=stream.cuda_stream)
    m.iterate(2000, 1)
    m.hmc(1, n_steps, step)                     # warm-up
    m.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    m.hmc(n_traj, n_steps, step)
    e1.record(stream)
    e1.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    W = wl.walkers_per_system
    acc = tot = 0
    for s in range(len(wl.systems)):
        _, _, c = m.walkers_state(s)
        acc += int(np.sum(c["hmc_accepted"]))
        tot += int(np.sum(c["hmc_trajectories"]))
    m.close()
    trajs = W * len(wl.systems) * n_traj
    flops = W * n_traj * n_steps * sum(hmc_flops_per_step(sp.chain_len) for sp in wl.systems)
    return {"walkers": W * len(wl.systems), "trajectories_per_walker": n_traj,
            "leapfrog_steps": n_steps, "step": step, "ms": sec * 1e3,
            "trajectories_per_s": trajs / sec, "leapfrog_steps_per_s": trajs * n_steps / sec,
            "acceptance": acc / max(1, tot), "fp64_tflops": flops / sec / 1e12,
            "fp64_peak_tflops": 78.6}


def differentiation_flops_per_config(chain_len, periodic=True):
    """Operations the energy forward + backward must perform for one stored configuration, each
    unordered non-bonded pair once (Newton's third law) and each bending / torsion term once.
    Forward: pair evaluation (13, +9 periodic) + accumulation 1; angle term 25 (two bond vectors
    6, two norms 12, dot product and 1 - cos 7).  Backward: pair evaluation again, force scalar
    kappa s (-12 s^6 + 6 C s^3) 5, force vector 3, added to both beads 6, coupling partial 1;
    angle term 25 + derivatives with respect to both bonds 24 + scattered to its beads 9."""
    n = int(np.sum(chain_len))
    m = len(chain_len)
    pairs = n * (n - 1) // 2 - (n - m)
    angles = sum(max(0, L - 2) for L in chain_len) + sum(max(0, L - 3) for L in chain_len)
    ev = 13 + (9 if periodic else 0)
    fwd = pairs * (ev + 1) + angles * 25
    bwd = pairs * (ev + 5 + 3 + 6 + 1) + angles * (25 + 24 + 9)
    return fwd, bwd


def differentiation_leg(stream, n_cfg=1_000_000, n_t=64, steps=3, warmup=1, sample_every=10):
    """The differentiation path on stored configurations of the cross-seeding mixture (4 x 9 +
    4 x 10 beads, periodic edge 25, bending + torsion): walkers of two short MUCA iterations are
    stored every `sample_every` sweeps until n_cfg FP32 configurations sit in HBM with their
    sampling weights ln W(E0).  One step = energy forward over all configurations, reweighted
    <E>_T and C_V(T) at n_t temperatures in [0.1, 1.0], the reweighting backward for
    L = sum_T (<E>_T + C_V(T)), and the energy backward (dE/dx and dE/dtheta).  Each kernel is
    timed with HIP events on the library's stream."""
    import torch

    import paper_1702_01770_amd as P
    import workloads
    wl = workloads.cross_seeding()
    sp = wl.systems[0]
    W, N = wl.walkers_per_system, sp.n_beads
    m = P.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=W,
                             stream=stream.cuda_stream)
    m.iterate(1000, 2)
    b, a, _ = m.weights(0)
    x = torch.empty((n_cfg, N, 3), dtype=torch.float32, device="cuda")
    e0 = np.empty(n_cfg)
    done = 0
    while done < n_cfg:
        m.sweep(sample_every)
        pos, e, _ = m.walkers_state(0)
        k = min(W, n_cfg - done)
        x[done:done + k].copy_(torch.from_numpy(pos[:k].astype(np.float32)))
        e0[done:done + k] = e[:k]
        done += k
    kb = np.clip(np.floor((e0 - sp.e_lo) / wl.bin_width).astype(np.int64), 0, sp.n_bins - 1)
    lnw0 = torch.tensor(-b[kb] * e0 + a[kb], dtype=torch.float64, device="cuda")
    theta = np.array([wl.c_lj[0, 1], wl.c_lj[1, 1], wl.k_bend, wl.k_tors])
    temps = np.linspace(0.1, 1.0, n_t)
    dev = "cuda"
    E = torch.empty(n_cfg, dtype=torch.float64, device=dev)
    mean = torch.empty(n_t, dtype=torch.float64, device=dev)
    cv = torch.empty_like(mean)
    mom = torch.empty(n_t, 3, dtype=torch.float64, device=dev)
    ws = torch.empty(P.reweight_workspace_bytes(n_cfg, n_t), dtype=torch.uint8, device=dev)
    g_mean = torch.ones(n_t, dtype=torch.float64, device=dev)
    g_cv = torch.ones(n_t, dtype=torch.float64, device=dev)
    gE = torch.empty_like(E)
    gx = torch.empty_like(x)
    gth = torch.empty(4, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    sid = stream.cuda_stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    tot = np.zeros(4)

    def one(record):
        if record:
            ev[0].record(stream)
        m.energy_fwd_ptr(0, x.data_ptr(), n_cfg, theta, E.data_ptr())
        if record:
            ev[1].record(stream)
        P.reweight_fwd(E.data_ptr(), lnw0.data_ptr(), n_cfg, temps, mean.data_ptr(),
                       cv.data_ptr(), mom.data_ptr(), ws.data_ptr(), ws.numel(), sid)
        if record:
            ev[2].record(stream)
        P.reweight_bwd(E.data_ptr(), lnw0.data_ptr(), n_cfg, temps, mom.data_ptr(),
                       g_mean.data_ptr(), g_cv.data_ptr(), gE.data_ptr(), sid)
        if record:
            ev[3].record(stream)
        m.energy_bwd_ptr(0, x.data_ptr(), n_cfg, theta, gE.data_ptr(), gx.data_ptr(),
                         gth.data_ptr())
        if record:
            ev[4].record(stream)
            ev[4].synchronize()
            for i in range(4):
                tot[i] += ev[i].elapsed_time(ev[i + 1])

    for _ in range(warmup):
        one(False)
    m.synchronize()
    for _ in range(steps):
        one(True)
    m.close()
    ms = tot / steps
    fwd, bwd = differentiation_flops_per_config(sp.chain_len)
    step_ms = float(ms.sum())
    return {"workload": f"{n_cfg} stored configurations of the cross-seeding mixture "
                        f"(4x9 + 4x10 beads, periodic L=25, bending + torsion), sampled every "
                        f"{sample_every} sweeps from 4096 walkers; {n_t} temperatures in [0.1, 1]",
            "steps": steps, "ms_per_step": step_ms,
            "configs_per_s": n_cfg / (step_ms / 1e3),
            "kernel_ms": {"energy_fwd": ms[0], "reweight_fwd": ms[1], "reweight_bwd": ms[2],
                          "energy_bwd": ms[3]},
            "algorithmic_flop_per_config": {"forward": fwd, "backward": bwd},
            "energy_fwd_tflops": fwd * n_cfg / (ms[0] / 1e3) / 1e12,
            "energy_bwd_tflops": bwd * n_cfg / (ms[3] / 1e3) / 1e12,
            "peak_tflops": PEAK_FP32_TFLOPS,
            "grad_theta": gth.cpu().tolist(),
            "mean_E_at_T": [float(mean[0]), float(mean[-1])]}


def cpu_baseline(wl, target_s: float = 15.0):
    """FP64 oracle on one host core: one walker of every system, sweeps sized to ~target_s."""
    import oracle
    import workloads
    oracle.build(force=False)
    pos0 = workloads.initial_positions(wl)
    walkers = []
    for s, sp in enumerate(wl.systems):
        sysd = oracle.System.from_workload(wl, s)
        walkers.append((oracle.Walker(sysd, pos0[s], s * wl.walkers_per_system, wl.seed),
                        oracle.Weights(sp.e_lo, wl.bin_width, sp.n_bins), sp))
    mv = oracle.move_params(wl)

    def sweep_all(n):
        moves = 0
        t0 = time.perf_counter()
        for w, W, sp in walkers:
            H = np.zeros(sp.n_bins, np.uint64)
            before = w.counters.moves
            w.run(W, mv, n, H)
            moves += w.counters.moves - before
        return moves, time.perf_counter() - t0

    m0, t0 = sweep_all(10)
    n = max(10, int(10 * target_s / max(t0, 1e-3)))
    m1, t1 = sweep_all(n)
    return dict(value=m1 / t1, unit="moves/s", cores=1, kind="oracle",
                sample=f"1 walker of each of the {len(wl.systems)} systems x {n} sweeps "
                       f"({m1} single-bead moves, {t1:.1f} s, flat weights)")


def copy_calibration(n_mib: int = 512, reps: int = 3):
    """Plain device-to-device copies of known size; their FETCH_SIZE / WRITE_SIZE counters scale
    the counters of the sweep kernel to bytes (see profiles/)."""
    import torch
    a = torch.ones(n_mib * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    return n_mib


def code_hash(files) -> str:
    """SHA-256 of the given sources with comments and whitespace removed, so that editing a
    comment does not void a measurement of the code."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in files:
        txt = open(os.path.join(ROOT, f)).read()
        txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)
        txt = re.sub(r"//[^\n]*", " ", txt)
        h.update(re.sub(r"\s+", " ", txt).strip().encode())
    return h.hexdigest()


def sweep_counters():
    """The committed rocprofv3 counter record of the sweep launch (HBM bytes, VALU instructions
    per launch), or None when the sweep kernel's code changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "sweep_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if code_hash(rec.get("sources", [])) != rec.get("sources_code_sha256"):
        return None
    return rec


def sweep_traffic():
    """HBM bytes per sweep launch from the committed counter record, or None (see above)."""
    rec = sweep_counters()
    return rec["bytes_per_launch"] if rec else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run 512 MiB device copies first (counter calibration)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--sweeps", type=int, default=100000, help="sweeps per MUCA iteration")
    ap.add_argument("--plain-sweeps", type=int, default=20000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-matched", action="store_true")
    ap.add_argument("--no-chain", action="store_true", help="skip the pivot leg")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiation leg")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper-systems leg")
    ap.add_argument("--no-hmc", action="store_true", help="skip the hybrid Monte Carlo leg")
    ap.add_argument("--paper-physics", default="",
                    help="comma-separated paper systems: only run their full MUCA + analysis")
    ap.add_argument("--physics-iters", type=int, default=1000)
    ap.add_argument("--physics-walkers", type=int, default=4096)
    ap.add_argument("--physics-ehi", type=float, default=None,
                    help="upper edge of the energy window (total energy) in the physics leg")
    ap.add_argument("--physics-reset", type=int, default=0,
                    help="clear the recursion's accumulated statistics every N iterations")
    ap.add_argument("--physics-hmc", type=int, default=0,
                    help="hybrid MC trajectories per walker and iteration in the physics leg")
    ap.add_argument("--diff-only", action="store_true",
                    help="run only the differentiation leg (profiling)")
    ap.add_argument("--diff-configs", type=int, default=1_000_000)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the launch plan given by --walkers-per-wave / --waves-per-block")
    ap.add_argument("--walkers-per-wave", type=int, default=0)
    ap.add_argument("--waves-per-block", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU (no multi-GPU path is implemented); --gpus must be 1"}))
        sys.exit(2)
    import workloads

    wl = workloads.batched_chains()
    st = make_stream()
    if args.calibrate_copy:
        copy_calibration()
    if args.paper_physics:
        print(json.dumps({"paper_physics": paper_physics_leg(
            st, args.paper_physics.split(","), iters=args.physics_iters,
            walkers=args.physics_walkers, hmc_traj=args.physics_hmc,
            reset_every=args.physics_reset, e_hi=args.physics_ehi,
            first=int(0.7 * args.physics_iters), block=max(1, args.physics_iters // 40))}))
        return
    if args.diff_only:
        print(json.dumps({"differentiation": differentiation_leg(st, args.diff_configs,
                                                                 steps=args.steps,
                                                                 warmup=args.warmup)}))
        return
    r = run_gpu(wl, wl.walkers_per_system, args.sweeps, args.steps, args.warmup, st,
                autotune=not args.no_autotune, walkers_per_wave=args.walkers_per_wave,
                waves_per_block=args.waves_per_block)
    sec = r["event_ms"] / 1e3
    value = r["moves"] / sec
    flops_per_step = sum(wl.walkers_per_system * args.sweeps * sp.n_beads *
                         algorithmic_flops_per_move(sp.n_beads) for sp in wl.systems)
    achieved = flops_per_step * args.steps / sec / 1e12
    out = {
        "metric": "MC moves/sec (batched vs plain, 1 GPU) at matched S(E) error vs FP64 oracle",
        "value": value, "unit": "moves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["event_ms"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 pair terms + f64 energy/weights", "data": "synthetic",
        "config": {"workload": "batched single chains: 32 seeded A/B sequences, N uniform in "
                               "13..55, 4096 walkers (128/system), FP32-split",
                   "sweeps_per_step": args.sweeps, "parallelism": "single GPU",
                   "launch_plan": r["plan"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": sweep_traffic()},
        "sweep_launch": {"launches": r["launches"],
                         "avg_ms": r["event_ms"] / r["launches"],
                         "algorithmic_flop_per_launch": flops_per_step * args.steps / r["launches"]},
        "acceptance": r["acc_rate"],
        "wall_s": r["wall_s"],
    }
    if not args.no_plain:
        rp = run_gpu(wl, 1, args.plain_sweeps, 1, 0, st, autotune=False)
        plain = rp["moves"] / (rp["event_ms"] / 1e3)
        out["plain"] = {"value": plain, "unit": "moves/s", "walkers_per_system": 1,
                        "sweeps": args.plain_sweeps}
        out["batched_over_plain"] = value / plain
    if not args.no_matched:
        out["matched_error"] = matched_error(st)
    if not args.no_chain:
        out["with_pivots"] = chain_moves_leg(wl, st)
    if not args.no_paper:
        out["paper_systems"] = paper_systems_leg(st)
    if not args.no_hmc:
        out["hybrid_mc"] = hmc_leg(st)
    if not args.no_diff:
        out["differentiation"] = differentiation_leg(st, args.diff_configs)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
