"""Benchmark: multicanonical (MUCA) trial moves per second on one MI355X.

Headline workload (synthetic stand-in for the paper's chains, see workloads.batched_chains): 32
single-chain AB systems with lengths drawn uniformly from 13..55 (~60 % A), 128 walkers per system
(4096 walkers), bin width 0.05 over [-4N, +N), FP32 pair arithmetic with FP64 energies / weights.
One step = one MUCA iteration: --sweeps sweeps of every walker followed by the Berg weight
update, replayed from a captured HIP graph (persistent sweep launches + update kernel).

Printed JSON line: value = single-bead trial moves per second over all walkers of that workload,
the roofline of its sweep kernel (algorithmic FP32/FP64 ALU operations per launch over the launch
time measured with HIP events on the library's stream), and beside it:
  * matched_error: the plain (one walker) and batched (4096 walkers sharing ln W) forms on the
    13-bead chain, each run until its entropy is as close to the FP64 oracle's reference as the
    oracle's own replicas get at that chain's budget (tests/golden/muca_c1_reference.json):
    moves/s and GPU time to that target for both forms;
  * configs: throughput of the aggregation (4 x 9 beads) and cross-seeding (76 beads) workloads
    and of the headline workload in FP64;
  * cpu_baseline: the FP64 oracle on the host cores (one core, median of five, and one process
    per core, pinned) running the same evolving-weight MUCA scheme on a bounded sample.
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
PEAK_FP64_TFLOPS = 78.6       # MI355X vector FP64 (published)


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


def rigid_flops(chain_len: int, n_beads: int, periodic: bool = True) -> float:
    """Operations of one rigid translation of a chain of chain_len beads among n_beads: every
    inter-chain pair of the moved chain evaluated before and after (13, +9 periodic, each), their
    difference and accumulation (2), plus the shift and the acceptance (60)."""
    pairs = chain_len * (n_beads - chain_len)
    return pairs * (2 * (13 + (9 if periodic else 0)) + 2) + 60


def workload_flops_per_sweep(wl, sp) -> float:
    """Algorithmic operations of one sweep of one walker of system sp: N single-bead moves and
    the rigid translations of a multi-chain system."""
    periodic = wl.box_kind == 2
    torsion = wl.k_tors != 0.0
    f = sp.n_beads * algorithmic_flops_per_move(sp.n_beads, len(sp.chain_len), periodic, torsion)
    if len(sp.chain_len) > 1 and wl.rigid_per_sweep:
        # the translated chain is drawn uniformly from the system's chains
        f += wl.rigid_per_sweep * float(np.mean([rigid_flops(n, sp.n_beads, periodic)
                                                 for n in sp.chain_len]))
    return f


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


def _grid_entropy(beta, alpha, e_lo, eps, k_lo, k_hi):
    """S_n(E) = beta_k E - alpha_k (Eq. 8) at the centres of bins [k_lo, k_hi), zero at the top."""
    k = np.arange(k_lo, k_hi)
    E = e_lo + (k + 0.5) * eps
    S = beta[k] * E - alpha[k]
    return S - S[-1]


def _aligned_error(S, S_ref, sigma, lo):
    """max over the converged grid points [lo, top) of |S - S_ref - c|, c the offset that
    minimises the sum of ((S - S_ref - c) / sigma)^2."""
    sl = slice(lo, len(S_ref) - 1)
    d = S[sl] - S_ref[sl]
    w = 1.0 / sigma[sl] ** 2
    c = float(np.sum(w * d) / np.sum(w))
    return float(np.max(np.abs(d - c)))


def matched_error(stream, plain_reps=16, plain_sweeps=100_000, max_plain_iters=20,
                  batched_walkers=4096, batched_sweeps=250, batched_reps=4,
                  max_batched_iters=50, eq_sweeps=300):
    """Plain vs batched form of MUCA at matched S(E) error on the 13-bead chain (FP64).

    Target: the aligned entropy error the FP64 oracle reaches at that chain's budget (one walker,
    ten iterations of 10^5 sweeps), as the median over its replicas, measured against a longer
    parallel-MUCA oracle reference on the grid range where that reference has converged; all of
    it is read from tests/golden/muca_c1_reference.json (written from the oracle only).
    Plain form: one walker, iterations of 10^5 sweeps; `plain_reps` independent replicas run
    side by side (one wave each), exactly the schedule of the oracle's replicas, and each stops
    the clock when its error first reaches the target (a replica trapped in compact states may
    never reach it; its time counts as infinite in the median).  Batched form: `batched_walkers`
    walkers sharing ln W, one replica after another: every walker first thermalises for
    `eq_sweeps` sweeps at W = 1 whose statistics are discarded (all walkers start from the
    straight chain, and with few sweeps per walker that start would bias the first histogram,
    which Berg's accumulation keeps weighting), then iterations of `batched_sweeps` sweeps per
    walker.  Times are GPU times of the thermalisation and the MUCA iterations (sweeps + weight
    update) from HIP events on the library's stream; the error checks run on the host in
    between."""
    import torch

    import paper_1702_01770_amd as P
    import workloads
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "muca_c1_reference.json")))
    rr = ref["reference"]
    S_ref, sigma = np.array(rr["S"]), np.array(rr["replica_sigma"])
    lo, target = rr["converged_from"], ref["target"]["delta_S"]
    k_lo, k_hi = ref["k_lo"], ref["k_hi"]
    wl0 = workloads.single_chain()
    sp = wl0.systems[0]
    N = sp.n_beads
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def one_iteration(m, sweeps):
        e0.record(stream)
        m.iterate(sweeps, 1)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / 1e3

    def thermalise(m, n_sys):
        if not eq_sweeps:
            return 0.0
        dt = one_iteration(m, eq_sweeps)
        zero = np.zeros(sp.n_bins)
        for r in range(n_sys):
            m.set_weights(r, zero, zero, zero)        # back to W = 1, statistics discarded
        return dt

    def errors(m, n_sys):
        out = []
        for r in range(n_sys):
            b, a, _ = m.weights(r)
            out.append(_aligned_error(_grid_entropy(b, a, sp.e_lo, wl0.bin_width, k_lo, k_hi),
                                      S_ref, sigma, lo))
        return out

    # plain: replicas as independent systems of one context, one walker each
    wl = workloads.single_chain()
    wl.systems = [sp] * plain_reps
    m = P.Muca.from_workload(wl, workloads.initial_positions(wl0) * plain_reps, walkers=1,
                             precision=0, seed=55_000_001, stream=stream.cuda_stream)
    hit, hit_it, plain_s, p_trace = [None] * plain_reps, [None] * plain_reps, [], []
    t_cum = 0.0
    for it in range(max_plain_iters):
        dt = one_iteration(m, plain_sweeps)
        t_cum += dt
        plain_s.append(dt)
        errs = errors(m, plain_reps)
        p_trace.append(float(np.median(errs)))
        for r, e in enumerate(errs):
            if hit[r] is None and e <= target:
                hit[r], hit_it[r] = t_cum, it + 1
        if all(h is not None for h in hit):
            break
    m.close()
    plain_rate = plain_sweeps * N / float(np.median(plain_s))
    reached = [h for h in hit if h is not None]
    censored = sorted(h if h is not None else float("inf") for h in hit)
    plain_median = float(np.median(censored))

    # batched: 4096 walkers sharing the weights of one system
    b_hit, b_it, b_rate, plan, b_traces = [], [], [], None, []
    for rep in range(batched_reps):
        m = P.Muca.from_workload(wl0, workloads.initial_positions(wl0), walkers=batched_walkers,
                                 precision=0, seed=56_000_001 + 1000 * rep,
                                 stream=stream.cuda_stream)
        m.autotune(probe_sweeps=20)           # restores the sampling state afterwards
        plan = m.launch_info()
        times, trace = [], []
        t_cum = thermalise(m, 1)
        for it in range(max_batched_iters):
            dt = one_iteration(m, batched_sweeps)
            t_cum += dt
            times.append(dt)
            e = errors(m, 1)[0]
            trace.append(e)
            if e <= target:
                b_hit.append(t_cum)
                b_it.append(it + 1)
                break
        b_traces.append(trace[:12])
        b_rate.append(batched_walkers * batched_sweeps * N / float(np.median(times)))
        m.close()
    out = {
        "system": "single 13-bead AB chain (workloads.single_chain), FP64, window [-52, 13)",
        "target": {"delta_S": target, "definition": "median aligned S(E) error of the FP64 "
                   "oracle's replicas at 1 walker x 10 iterations x 1e5 sweeps, against a "
                   "16-run parallel-MUCA oracle reference, on bins from E = "
                   f"{rr['converged_e']:.3f} to the window top"},
        "plain": {"walkers": 1, "sweeps_per_iteration": plain_sweeps, "replicas": plain_reps,
                  "max_iterations": max_plain_iters, "moves_per_s": plain_rate,
                  "reached": len(reached),
                  "time_to_target_s": plain_median if np.isfinite(plain_median) else None,
                  "time_to_target_s_of_those_reaching": float(np.median(reached))
                  if reached else None,
                  "time_at_oracle_budget_s": 10 * float(np.median(plain_s)),
                  "iterations_to_target": float(np.median([i for i in hit_it if i]))
                  if reached else None, "median_error_by_iteration": p_trace},
        "batched": {"walkers": batched_walkers, "sweeps_per_walker_per_iteration": batched_sweeps,
                    "replicas": batched_reps, "moves_per_s": float(np.median(b_rate)),
                    "reached": len(b_hit),
                    "time_to_target_s": float(np.median(b_hit)) if b_hit else None,
                    "iterations_to_target": float(np.median(b_it)) if b_it else None,
                    "error_by_iteration": b_traces, "launch_plan": plan},
        "thermalisation_sweeps": eq_sweeps,
    }
    if b_hit:
        # the plain form's median time to the target; when fewer than half of its replicas get
        # there within max_plain_iters, the time of the oracle's own budget (ten iterations, at
        # which half of the oracle's replicas are within the target by its definition)
        t_plain = out["plain"]["time_to_target_s"] or out["plain"]["time_at_oracle_budget_s"]
        out["time_ratio_plain_over_batched"] = t_plain / out["batched"]["time_to_target_s"]
    out["moves_per_s_ratio_batched_over_plain"] = out["batched"]["moves_per_s"] / plain_rate
    return out


def config_leg(name, wl, sweeps, steps, warmup, stream, precision=None):
    """Throughput of one workload: single-bead moves/s over all walkers (plus rigid moves) and
    the algorithmic operations per second against the vector peak of the arithmetic it runs in
    (FP32 pair terms: 157.3 TFLOP/s; FP64: 78.6), autotuned, timed over `steps` MUCA
    iterations after `warmup`."""
    import dataclasses
    if precision is not None:
        wl = dataclasses.replace(wl, precision=precision,
                                 resync_sweeps=wl.resync_sweeps if precision else 0)
    r = run_gpu(wl, wl.walkers_per_system, sweeps, steps, warmup, stream)
    sec = r["event_ms"] / 1e3
    W = wl.walkers_per_system
    flops = sum(W * sweeps * steps * workload_flops_per_sweep(wl, sp) for sp in wl.systems)
    rigid = sum(W * sweeps * steps * wl.rigid_per_sweep for sp in wl.systems
                if len(sp.chain_len) > 1)
    fp32 = wl.precision == 1
    peak = PEAK_FP32_TFLOPS if fp32 else PEAK_FP64_TFLOPS
    achieved = flops / sec / 1e12
    return {"workload": name, "walkers": W * len(wl.systems),
            "precision": "f32 pair terms + f64 energy/weights" if fp32 else "f64",
            "sweeps_per_step": sweeps, "steps": steps, "ms_per_step": r["event_ms"] / steps,
            "moves_per_s": r["moves"] / sec, "rigid_moves_per_s": rigid / sec,
            "acceptance": r["acc_rate"],
            "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                         "frac": achieved / peak},
            "sweep_launch": {"launches": r["launches"], "avg_ms": r["event_ms"] / r["launches"]},
            "launch_plan": r["plan"]}


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


def paper_physics_leg(stream, names, iters=1000, walkers=4096, first=700, block=25):
    """Full multicanonical runs of the paper's example systems as in Sec. 4: `walkers` walkers
    share the paper's sweeps per iteration, `iters` Berg iterations, then the
    microcanonical analysis (Eqs. 4-8) of iterations [first, iters) in blocks of `block`:
    Maxwell construction on beta(eps), latent heat and free-energy barrier per monomer, and
    whether the caloric curve bends back (a region of negative microcanonical specific heat).
    Flatness per iteration as the paper judges it: c_var < 5 % and peaks within 20 %."""
    import paper_1702_01770_amd as P
    import workloads
    out = {}
    for name in names:
        wl = workloads.paper_system(name, walkers=walkers)
        sp = wl.systems[0]
        sweeps = -(-PAPER_SWEEPS_PER_ITERATION[name] // walkers)
        m = P.Muca.from_workload(wl, workloads.initial_positions(wl),
                                 walkers=wl.walkers_per_system, stream=stream.cuda_stream)
        m.autotune(probe_sweeps=20)
        B = np.zeros((iters, sp.n_bins))
        A = np.zeros((iters, sp.n_bins))
        t0 = time.perf_counter()
        for it in range(iters):
            m.iterate(sweeps, 1)
            B[it], A[it], _ = m.weights(0)
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
               "walkers": walkers,
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


def _cpu_muca_sample(args):
    """One oracle process: one walker of every system of the workload (walker id `walker`), run
    through `iters` MUCA iterations of `sweeps` sweeps with a Berg update of each system's
    weights after every iteration (the evolving-weight scheme the GPU leg times).  Optionally
    pinned to one core.  Returns (single-bead moves, seconds)."""
    walker, iters, sweeps, cpu = args
    if cpu is not None:
        os.sched_setaffinity(0, {cpu})
    import oracle
    import workloads
    wl = workloads.batched_chains()
    pos0 = workloads.initial_positions(wl)
    mv = oracle.move_params(wl)
    runs = []
    for s, sp in enumerate(wl.systems):
        sysd = oracle.System.from_workload(wl, s)
        runs.append((oracle.Walker(sysd, pos0[s], s * wl.walkers_per_system + walker, wl.seed),
                     oracle.Weights(sp.e_lo, wl.bin_width, sp.n_bins), sp))
    moves = 0
    t0 = time.perf_counter()
    for _ in range(iters):
        for w, W, sp in runs:
            H = np.zeros(sp.n_bins, np.uint64)
            before = w.counters.moves
            w.run(W, mv, sweeps, H)
            moves += w.counters.moves - before
            W.berg_update(H)
    return moves, time.perf_counter() - t0


def cpu_baseline(target_s: float = 4.0, repeats: int = 5, max_procs: int = 16):
    """The FP64 oracle as it stands on the host: (a) one core, `repeats` runs of a sample sized
    to about target_s seconds, median rate; (b) one process per core (at most max_procs, the
    host share of one GPU), each pinned to its own core with its own walker ids, the paper's
    rank-per-core parallel scheme (Sec. 2.2) without the histogram merge; summed rate."""
    import multiprocessing as mp
    import oracle
    oracle.build(force=False)
    iters = 3
    m0, t0 = _cpu_muca_sample((0, 1, 20, None))
    sweeps = max(20, int(20 * target_s / max(t0, 1e-3) / iters))
    single = [_cpu_muca_sample((0, iters, sweeps, None)) for _ in range(repeats)]
    rates = [mv / t for mv, t in single]
    cpus = sorted(os.sched_getaffinity(0))
    P = min(len(cpus), max_procs)
    ctx = mp.get_context("spawn")
    with ctx.Pool(P) as pool:
        par = pool.map(_cpu_muca_sample, [(p + 1, iters, sweeps, cpus[p]) for p in range(P)])
    summed = sum(mv / t for mv, t in par)
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=summed, unit="moves/s", cores=P, kind="oracle",
                sample=f"each process: 1 walker of each of the 32 systems of the headline "
                       f"workload, {iters} MUCA iterations x {sweeps} sweeps with a Berg "
                       f"update after each ({single[0][0]} single-bead moves, about "
                       f"{single[0][1]:.1f} s); {P} processes pinned one per core",
                single_core={"moves_per_s_median": float(np.median(rates)),
                             "runs": [float(r) for r in rates]},
                per_process_moves_per_s=[float(mv / t) for mv, t in par],
                nproc=os.cpu_count(), affinity_cpus=len(cpus), cpu_model=model)


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


def flop_calibration(n: int = 1 << 26, reps: int = 3):
    """Plain FP32 and FP64 elementwise multiplies of known size (one multiply per element): their
    SQ_INSTS_VALU_MUL_F32 / _F64 counters give the number of element operations one counted
    instruction stands for (64 for one wave64 instruction without packing), the factor that
    turns the sweep kernel's instruction counters into FLOP (see profiles/)."""
    import torch
    for dt in (torch.float32, torch.float64):
        a = torch.full((n,), 1.0001, dtype=dt, device="cuda")
        for _ in range(reps):
            torch.mul(a, 1.0001, out=a)
    torch.cuda.synchronize()
    return n


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


LEGS = ("matched", "configs", "pivots", "paper", "hmc", "diff", "cpu")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run 512 MiB device copies first (counter calibration)")
    ap.add_argument("--calibrate-flops", action="store_true",
                    help="run FP32 and FP64 elementwise multiplies first (counter calibration)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--sweeps", type=int, default=100000, help="sweeps per MUCA iteration")
    ap.add_argument("--skip", default="", help="comma-separated legs to skip: " + ",".join(LEGS))
    ap.add_argument("--only", default="",
                    help="run only this leg (main, matched, c3, c4, c2_fp64, "
                         "c2_fp32_same_schedule, pivots, paper, hmc, diff, cpu) and print it "
                         "alone (profiling)")
    ap.add_argument("--paper-physics", default="",
                    help="comma-separated paper systems: only run their full MUCA + analysis")
    ap.add_argument("--physics-iters", type=int, default=1000)
    ap.add_argument("--physics-walkers", type=int, default=4096)
    ap.add_argument("--diff-configs", type=int, default=1_000_000)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the launch plan given by --walkers-per-wave / --waves-per-block")
    ap.add_argument("--walkers-per-wave", type=int, default=0)
    ap.add_argument("--waves-per-block", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU (no multi-GPU path is "
                                   "implemented); --gpus must be 1"}))
        sys.exit(2)
    import workloads

    wl = workloads.batched_chains()
    st = make_stream()
    if args.calibrate_copy:
        copy_calibration()
    if args.calibrate_flops:
        flop_calibration()
    if args.paper_physics:
        print(json.dumps({"paper_physics": paper_physics_leg(
            st, args.paper_physics.split(","), iters=args.physics_iters,
            walkers=args.physics_walkers, first=int(0.7 * args.physics_iters),
            block=max(1, args.physics_iters // 40))}))
        return
    configs = {
        "c3": lambda: config_leg("aggregation: 4 x 9 beads, periodic cube L=20, 1024 walkers, "
                                 "FP32-split, one rigid translation per sweep",
                                 workloads.aggregation(), 10000, 3, 1, st),
        "c4": lambda: config_leg("cross-seeding: 4 x 9 + 4 x 10 beads, periodic cube L=25, "
                                 "bending + torsion, 4096 walkers, FP32-split, one rigid "
                                 "translation per sweep", workloads.cross_seeding(), 10000, 3,
                                 1, st),
        "c2_fp64": lambda: config_leg("batched single chains (the headline workload) in FP64",
                                      wl, 20000, 3, 1, st, precision=0),
        # the same schedule in the FP32-split mode: the FP64 line's counterpart at the same
        # weights' history and hence acceptance (the headline runs longer iterations)
        "c2_fp32_same_schedule": lambda: config_leg(
            "batched single chains (the headline workload), FP32-split, on the FP64 line's "
            "schedule", wl, 20000, 3, 1, st),
    }
    single = dict(configs, matched=lambda: matched_error(st),
                  pivots=lambda: chain_moves_leg(wl, st), paper=lambda: paper_systems_leg(st),
                  hmc=lambda: hmc_leg(st),
                  diff=lambda: differentiation_leg(st, args.diff_configs, steps=args.steps,
                                                   warmup=args.warmup),
                  cpu=lambda: cpu_baseline())
    if args.only and args.only != "main":
        print(json.dumps({args.only: single[args.only]()}))
        return
    skip = set(x for x in args.skip.split(",") if x)
    r = run_gpu(wl, wl.walkers_per_system, args.sweeps, args.steps, args.warmup, st,
                autotune=not args.no_autotune, walkers_per_wave=args.walkers_per_wave,
                waves_per_block=args.waves_per_block)
    sec = r["event_ms"] / 1e3
    value = r["moves"] / sec
    flops_per_step = sum(wl.walkers_per_system * args.sweeps * workload_flops_per_sweep(wl, sp)
                         for sp in wl.systems)
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
    if args.only == "main":
        print(json.dumps(out))
        return
    if "matched" not in skip:
        out["matched_error"] = single["matched"]()
    if "configs" not in skip:
        out["configs"] = {k: f() for k, f in configs.items()}
    if "pivots" not in skip:
        out["with_pivots"] = single["pivots"]()
    if "paper" not in skip:
        out["paper_systems"] = single["paper"]()
    if "hmc" not in skip:
        out["hybrid_mc"] = single["hmc"]()
    if "diff" not in skip:
        out["differentiation"] = differentiation_leg(st, args.diff_configs)
    if "cpu" not in skip:
        out["cpu_baseline"] = single["cpu"]()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
