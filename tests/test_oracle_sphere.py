"""Pins of the oracle's steric sphere (the container of the paper's simulations, Sec. 4): a trial
move that would take a bead outside the sphere is rejected.  Checked against the exact radial
law of the middle bead of a free 3-bead chain, the no-box limit of a huge sphere, and the
invariant that no bead ever leaves."""
import dataclasses

import numpy as np

import workloads

CP = workloads.C_LJ_PAPER


def _no_energy_three_beads(orc, radius):
    return orc.System([3], np.zeros(3, np.uint8), CP, k_intra=0.0, k_inter=0.0, k_bend=0.0,
                      box_kind=workloads.BOX_SPHERE, box_len=radius)


def test_free_three_bead_chain_middle_radial_law(orc):
    """Without interactions every allowed configuration is equally likely under the symmetric
    moves, i.e. bead 0 uniform in space and both bonds uniform on the unit sphere, restricted to
    the ball.  Given the middle bead at distance d from the centre, each end bead is inside with
    probability f(d) = clip((1 + (R^2 - d^2 - 1) / (2 d)) / 2, 0, 1) (the part of its unit
    sphere inside the ball), so the middle bead's radial density is d^2 f(d)^2 on [0, R]."""
    R = 2.0
    s = _no_energy_three_beads(orc, R)
    W = orc.Weights(-1.0, 0.05, 40)               # E = 0 always lies in the window
    mv = dict(crank_max=np.pi / 3, cap_rho=0.8, trans_max=0.0, rigid_per_sweep=0)
    edges = np.linspace(0.0, R, 11)
    n_q = 400_000
    d = (np.arange(n_q) + 0.5) * (R / n_q)
    f = np.clip((1.0 + (R * R - d * d - 1.0) / (2.0 * d)) / 2.0, 0.0, 1.0)
    dens = d * d * f * f
    p_exact = np.array([dens[(d >= a) & (d < b)].sum() for a, b in zip(edges[:-1], edges[1:])])
    p_exact /= p_exact.sum()
    start = np.array([[-1.0, 0, 0], [0, 0, 0], [1, 0, 0]])
    fr = []
    for wid in range(8):
        w = orc.Walker(s, start, wid, 91)
        H = np.zeros(W.n_bins, np.uint64)
        w.run(W, mv, 300, H)                      # burn-in
        r = np.empty(12000)
        for i in range(r.size):
            w.run(W, mv, 1, H)
            r[i] = np.linalg.norm(w.pos[1])
        assert np.max(np.linalg.norm(w.pos, axis=1)) <= R
        fr.append(np.histogram(r, bins=edges)[0] / r.size)
        assert w.counters.accepted < w.counters.moves          # the wall rejected moves
    fr = np.array(fr)
    m, se = fr.mean(axis=0), fr.std(axis=0, ddof=1) / np.sqrt(len(fr))
    z = (m - p_exact) / np.maximum(se, 1e-12)
    assert np.all(np.abs(z) < 5.0), (m, p_exact, z)
    # the law is far from the unconfined one (uniform middle bead): the outer shell is depleted
    assert p_exact[-1] < 0.5 * (1.0 - (edges[-2] / R) ** 3)


def _run(orc, wl, n_sweeps, walker=0, log=None, pos0=None):
    sp = wl.systems[0]
    s = orc.System.from_workload(wl)
    pos0 = workloads.initial_positions(wl)[0] if pos0 is None else pos0
    w = orc.Walker(s, pos0, walker, wl.seed)
    H = np.zeros(sp.n_bins, np.uint64)
    w.run(orc.Weights(sp.e_lo, wl.bin_width, sp.n_bins), orc.move_params(wl), n_sweeps, H,
          accept_log=log)
    return w, H


def test_huge_sphere_is_no_box(orc):
    """A sphere far larger than any excursion never rejects: the trajectory equals the one
    without a box move for move."""
    base = workloads.confined(radius=6.0)
    far = dataclasses.replace(base, box_len=1.0e6)
    free = dataclasses.replace(base, box_kind=workloads.BOX_NONE, box_len=0.0)
    n = 300
    pos0 = workloads.initial_positions(base)[0]
    la = np.zeros(n * 18, np.uint8)
    lb = np.zeros(n * 18, np.uint8)
    wa, ha = _run(orc, far, n, log=la, pos0=pos0)
    wb, hb = _run(orc, free, n, log=lb, pos0=pos0)
    assert np.array_equal(la, lb) and np.array_equal(ha, hb)
    assert np.array_equal(wa.pos, wb.pos) and wa.energy == wb.energy
    assert wa.counters.rigid_accepted == wb.counters.rigid_accepted


def test_tight_sphere_keeps_every_bead_inside(orc):
    """Two 9-bead chains in a sphere of radius 6 (they span 8 when straight): after many single-
    bead and rigid moves no bead is outside, while the unconfined run leaves it."""
    wl = workloads.confined(radius=6.0)
    free = dataclasses.replace(wl, box_kind=workloads.BOX_NONE, box_len=0.0)
    for walker in range(3):
        w, H = _run(orc, wl, 3000, walker)
        assert np.max(np.linalg.norm(w.pos, axis=1)) <= 6.0
        assert int(H.sum()) == w.counters.moves + w.counters.rigid_moves
        wf, _ = _run(orc, free, 3000, walker, pos0=workloads.initial_positions(wl)[0])
        assert np.max(np.linalg.norm(wf.pos, axis=1)) > 6.0
