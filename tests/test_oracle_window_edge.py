"""Pins of the reference's window-edge reading: a walker whose running energy lies at most
edge_tol outside the energy window (what reduced-precision accumulation can leave at an edge)
continues from the edge bin on that side; further outside, or without a tolerance, it is
refused; inside the window the tolerance changes nothing."""
import numpy as np
import pytest

import oracle
import workloads


def _coil(wl, s, sp):
    """A random coil: the initial chain after 200 canonical sweeps at T = 0.7 (from the
    straight start nearly every move raises the energy)."""
    W = oracle.Weights(sp.e_lo, wl.bin_width, sp.n_bins, np.full(sp.n_bins, 1 / 0.7),
                       np.zeros(sp.n_bins))
    w = oracle.Walker(s, workloads.initial_positions(wl)[0], 7, wl.seed)
    w.run(W, oracle.move_params(wl), 200, np.zeros(sp.n_bins, np.uint64))
    return w.pos.copy()


def _setup(offset, side):
    wl = workloads.single_chain()
    sp = wl.systems[0]
    s = oracle.System.from_workload(wl)
    pos = _coil(wl, s, sp)
    top = sp.e_lo + sp.n_bins * wl.bin_width
    e_start = top + offset if side == "top" else sp.e_lo - offset
    return wl, sp, s, pos, e_start


@pytest.mark.parametrize("side", ["top", "bottom"])
def test_start_within_tolerance_counts_in_the_edge_bin(side):
    wl, sp, s, pos, e_start = _setup(5e-4, side)
    K = sp.n_bins
    W = oracle.Weights(sp.e_lo, wl.bin_width, K, edge_tol=1e-3)      # flat weights
    w = oracle.Walker(s, pos, 0, wl.seed)
    w.energy = e_start
    H = np.zeros(K, np.uint64)
    n = 4 * sp.n_beads
    log = np.zeros(n, np.uint8)
    w.run(W, oracle.move_params(wl), 4, H, accept_log=log)
    assert int(H.sum()) == n                         # one count per trial move
    # flat weights: a move is accepted iff it ends inside the window, so until the first
    # accepted move the walker stays outside and each move counts in the edge bin
    edge = K - 1 if side == "top" else 0
    first = int(np.argmax(log)) if log.any() else n
    assert first >= 0 and int(H[edge]) >= max(1, first)
    assert log.any(), "no move entered the window"
    top = sp.e_lo + K * wl.bin_width
    assert sp.e_lo <= w.energy < top                 # it ends inside


@pytest.mark.parametrize("side", ["top", "bottom"])
def test_beyond_tolerance_or_without_it_is_refused(side):
    for offset, tol in ((5e-4, 0.0), (2e-3, 1e-3)):
        wl, sp, s, pos, e_start = _setup(offset, side)
        W = oracle.Weights(sp.e_lo, wl.bin_width, sp.n_bins, edge_tol=tol)
        w = oracle.Walker(s, pos, 0, wl.seed)
        w.energy = e_start
        with pytest.raises(ValueError):
            w.run(W, oracle.move_params(wl), 1, np.zeros(sp.n_bins, np.uint64))


def test_tolerance_changes_nothing_inside_the_window():
    wl = workloads.single_chain()
    sp = wl.systems[0]
    s = oracle.System.from_workload(wl)
    pos = workloads.initial_positions(wl)[0]
    beta = np.full(sp.n_bins, 1 / 0.7)
    out = []
    for tol in (0.0, 1e-3):
        W = oracle.Weights(sp.e_lo, wl.bin_width, sp.n_bins, beta, np.zeros(sp.n_bins),
                           edge_tol=tol)
        w = oracle.Walker(s, pos, 0, wl.seed)
        H = np.zeros(sp.n_bins, np.uint64)
        log = np.zeros(300 * sp.n_beads, np.uint8)
        w.run(W, oracle.move_params(wl), 300, H, accept_log=log)
        out.append((log, H, w.pos.copy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][2], out[1][2])
