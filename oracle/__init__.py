"""FP64 reference oracle for the multicanonical AB-chain sampler -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of `bench.py` may import this
package.  The product library (`paper_1702_01770_amd`) never imports it and shares no code with
it; the two meet only in the seeded input generators of `workloads`.

Parts:
  * `muca_oracle.c` (built to `liboracle.so` with gcc, no FMA contraction): Philox4x32-10,
    the energy of Eqs. (1)-(3), the single-bead moves, the MUCA Metropolis run of Sec. 2.2,
    Berg's weight recursion, the flatness statistics and the energy gradients;
  * `analysis.py`: the microcanonical analysis of Eqs. (4)-(8) (numpy, FP64);
  * `reweight.py`: canonical reweighting of stored MUCA samples and its parameter gradients
    (numpy, FP64).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "muca_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (serial FP64, -ffp-contract=off, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _System(C.Structure):
    _fields_ = [("n_beads", C.c_int32), ("n_chains", C.c_int32), ("n_types", C.c_int32),
                ("box_kind", C.c_int32), ("chain_start", C.POINTER(C.c_int32)),
                ("type", C.POINTER(C.c_uint8)), ("c_lj", C.POINTER(C.c_double)),
                ("k_intra", C.c_double), ("k_inter", C.c_double), ("k_bend", C.c_double),
                ("k_tors", C.c_double), ("box_len", C.c_double)]


class _Weights(C.Structure):
    _fields_ = [("e_lo", C.c_double), ("bin_width", C.c_double), ("n_bins", C.c_int32),
                ("beta", C.POINTER(C.c_double)), ("alpha", C.POINTER(C.c_double)),
                ("edge_tol", C.c_double)]


class _Moves(C.Structure):
    _fields_ = [("crank_max", C.c_double), ("cap_rho", C.c_double), ("trans_max", C.c_double),
                ("rigid_per_sweep", C.c_int32), ("pivot_per_sweep", C.c_int32),
                ("pivot_max", C.c_double), ("rotate_per_sweep", C.c_int32),
                ("rotate_max", C.c_double)]


class _Counters(C.Structure):
    _fields_ = [("moves", C.c_int64), ("accepted", C.c_int64), ("rigid_moves", C.c_int64),
                ("rigid_accepted", C.c_int64), ("window_rejects", C.c_int64),
                ("max_drift", C.c_double), ("pivot_moves", C.c_int64),
                ("pivot_accepted", C.c_int64), ("rot_moves", C.c_int64),
                ("rot_accepted", C.c_int64)]


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.orc_philox_many.argtypes = [C.c_int64, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                      C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_energy.restype = C.c_double
        L.orc_energy.argtypes = [C.POINTER(_System), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_run.restype = C.c_int
        L.orc_run.argtypes = [C.POINTER(_System), C.POINTER(_Weights), C.POINTER(_Moves),
                              C.c_uint64, C.c_uint32, C.POINTER(C.c_uint64),
                              C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int64,
                              C.POINTER(C.c_uint64), C.POINTER(C.c_uint8), C.c_int64, C.c_int64,
                              C.POINTER(_Counters)]
        L.orc_berg_update.argtypes = [C.c_int32, C.c_double, C.c_double, C.POINTER(C.c_uint64),
                                      C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.c_double, C.c_double]
        L.orc_flatness.argtypes = [C.c_int32, C.POINTER(C.c_uint64), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32)]
        L.orc_energy_many.argtypes = [C.POINTER(_System), C.c_int64, C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]
        L.orc_energy_grad.argtypes = [C.POINTER(_System), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]
        _lib = L
    return _lib


# ------------------------------------------------------------------------------------------
# Philox
# ------------------------------------------------------------------------------------------
def philox(k0, k1, ctr) -> np.ndarray:
    """Philox4x32-10 blocks: k0, k1 broadcast to ctr.shape[:-1]; ctr [..., 4] uint32."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32)
    shp = ctr.shape[:-1]
    n = int(np.prod(shp)) if shp else 1
    kk0 = np.ascontiguousarray(np.broadcast_to(np.asarray(k0, dtype=np.uint32), shp).reshape(n))
    kk1 = np.ascontiguousarray(np.broadcast_to(np.asarray(k1, dtype=np.uint32), shp).reshape(n))
    out = np.empty((n, 4), dtype=np.uint32)
    lib().orc_philox_many(n, _p(kk0, C.c_uint32), _p(kk1, C.c_uint32),
                          _p(ctr.reshape(n, 4), C.c_uint32), _p(out, C.c_uint32))
    return out.reshape(shp + (4,))


# ------------------------------------------------------------------------------------------
# Systems
# ------------------------------------------------------------------------------------------
class System:
    """A system (chains, letters, couplings, box) in the layout the C oracle reads."""

    def __init__(self, chain_len, types, c_lj, k_intra=4.0, k_inter=4.0, k_bend=0.25,
                 k_tors=0.0, box_kind=0, box_len=0.0):
        self.chain_len = [int(x) for x in chain_len]
        self.chain_start = np.ascontiguousarray(np.concatenate([[0], np.cumsum(self.chain_len)]),
                                                dtype=np.int32)
        self.types = np.ascontiguousarray(types, dtype=np.uint8)
        self.c_lj = np.ascontiguousarray(c_lj, dtype=np.float64)
        self.n_beads = int(self.chain_start[-1])
        assert self.types.shape == (self.n_beads,)
        self._s = _System(self.n_beads, len(self.chain_len), int(self.c_lj.shape[0]),
                          int(box_kind), _p(self.chain_start, C.c_int32), _p(self.types, C.c_uint8),
                          _p(self.c_lj, C.c_double), float(k_intra), float(k_inter), float(k_bend),
                          float(k_tors), float(box_len))

    @classmethod
    def from_workload(cls, wl, sys_index: int = 0, c_lj=None, k_bend=None, k_tors=None):
        sp = wl.systems[sys_index]
        return cls(sp.chain_len, sp.types, wl.c_lj if c_lj is None else c_lj, wl.k_lj_intra,
                   wl.k_lj_inter, wl.k_bend if k_bend is None else k_bend,
                   wl.k_tors if k_tors is None else k_tors, wl.box_kind, wl.box_len)

    def energy(self, pos) -> float:
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        return lib().orc_energy(C.byref(self._s), _p(pos, C.c_double), None, None)

    def energy_many(self, pos) -> np.ndarray:
        """Energies of configurations pos [n_cfg, N, 3]."""
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        out = np.empty(pos.shape[0])
        lib().orc_energy_many(C.byref(self._s), pos.shape[0], _p(pos, C.c_double),
                              _p(out, C.c_double))
        return out

    def energy_parts(self, pos):
        """(E, [bend, torsion, intra LJ, inter LJ], sum of |terms|)."""
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        parts = np.zeros(4)
        scale = C.c_double(0)
        e = lib().orc_energy(C.byref(self._s), _p(pos, C.c_double), _p(parts, C.c_double),
                             C.byref(scale))
        return e, parts, scale.value

    def energy_grad(self, pos):
        """(E, dE/dx [N,3], dE/dtheta [4]) with theta = (C_AB, C_BB, kappa_bend, kappa_tors)."""
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        g = np.zeros((self.n_beads, 3))
        gt = np.zeros(4)
        e = C.c_double(0)
        lib().orc_energy_grad(C.byref(self._s), _p(pos, C.c_double), C.byref(e),
                              _p(g, C.c_double), _p(gt, C.c_double))
        return e.value, g, gt


class Weights:
    """ln W(E) = -beta_k E + alpha_k on bins of width eps above e_lo (Eq. 8).  edge_tol > 0: a
    walker whose starting energy lies at most edge_tol outside the window starts in the edge bin
    on that side instead of being refused (the window-edge reading for energies left just outside
    by reduced-precision accumulation)."""

    def __init__(self, e_lo, bin_width, n_bins, beta=None, alpha=None, g=None, beta_min=0.0,
                 beta_max=0.0, edge_tol=0.0):
        self.beta_min, self.beta_max = float(beta_min), float(beta_max)
        self.edge_tol = float(edge_tol)
        self.e_lo = float(e_lo)
        self.bin_width = float(bin_width)
        self.n_bins = int(n_bins)
        self.beta = np.zeros(n_bins) if beta is None else np.array(beta, dtype=np.float64)
        self.alpha = np.zeros(n_bins) if alpha is None else np.array(alpha, dtype=np.float64)
        self.g = np.zeros(n_bins) if g is None else np.array(g, dtype=np.float64)

    def _c(self):
        return _Weights(self.e_lo, self.bin_width, self.n_bins, _p(self.beta, C.c_double),
                        _p(self.alpha, C.c_double), self.edge_tol)

    def berg_update(self, hist):
        hist = np.ascontiguousarray(hist, dtype=np.uint64)
        lib().orc_berg_update(self.n_bins, self.e_lo, self.bin_width, _p(hist, C.c_uint64),
                              _p(self.beta, C.c_double), _p(self.alpha, C.c_double),
                              _p(self.g, C.c_double), self.beta_min, self.beta_max)

    def copy(self):
        return Weights(self.e_lo, self.bin_width, self.n_bins, self.beta, self.alpha, self.g,
                       self.beta_min, self.beta_max, self.edge_tol)


def flatness(hist):
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    cv, pk = C.c_double(0), C.c_double(0)
    lo, hi = C.c_int32(0), C.c_int32(0)
    lib().orc_flatness(len(hist), _p(hist, C.c_uint64), C.byref(cv), C.byref(pk), C.byref(lo),
                       C.byref(hi))
    return cv.value, pk.value, lo.value, hi.value


class Walker:
    """State of one Markov chain: coordinates, running energy, sweep counter, stream id."""

    def __init__(self, system: System, pos, walker_id: int, seed: int):
        self.system = system
        self.pos = np.array(pos, dtype=np.float64, order="C")
        self.energy = system.energy(self.pos)
        self.sweeps = 0
        self.walker_id = int(walker_id)
        self.seed = int(seed)
        self.counters = _Counters()

    def run(self, weights: Weights, moves: dict, n_sweeps: int, hist, accept_log=None,
            check_every: int = 0):
        mv = _Moves(moves["crank_max"], moves["cap_rho"], moves["trans_max"],
                    moves["rigid_per_sweep"], moves.get("pivot_per_sweep", 0),
                    moves.get("pivot_max", 0.0), moves.get("rotate_per_sweep", 0),
                    moves.get("rotate_max", 0.0))
        sc = C.c_uint64(self.sweeps)
        e = C.c_double(self.energy)
        w = weights._c()
        if accept_log is None:
            logp, cap = None, 0
        else:
            logp, cap = _p(accept_log, C.c_uint8), len(accept_log)
        rc = lib().orc_run(C.byref(self.system._s), C.byref(w), C.byref(mv), self.seed,
                           self.walker_id, C.byref(sc), _p(self.pos, C.c_double), C.byref(e),
                           int(n_sweeps), _p(hist, C.c_uint64), logp, cap, int(check_every),
                           C.byref(self.counters))
        if rc != 0:
            raise ValueError("walker energy outside the window")
        self.sweeps = sc.value
        self.energy = e.value


def move_params(wl) -> dict:
    return dict(crank_max=wl.crank_max, cap_rho=wl.cap_rho, trans_max=wl.trans_max,
                rigid_per_sweep=wl.rigid_per_sweep if wl.rigid_per_sweep else 0,
                pivot_per_sweep=wl.pivot_per_sweep, pivot_max=wl.pivot_max,
                rotate_per_sweep=wl.rotate_per_sweep, rotate_max=wl.rotate_max)


def muca(wl, sys_index: int = 0, n_iter: Optional[int] = None, n_sweeps: Optional[int] = None,
         walkers: Optional[int] = None, walker_offset: int = 0, seed: Optional[int] = None):
    """Parallel MUCA iteration scheme of Sec. 2.2 (Fig. 2) for one system, run serially:
    all walkers start from the same weights, their histograms are summed after every iteration
    and Berg's recursion produces the next weights.  Returns per-iteration arrays
    beta[n], alpha[n], g[n] (after the update of iteration n) and hist[n]."""
    import workloads
    sysd = System.from_workload(wl, sys_index)
    sp = wl.systems[sys_index]
    n_iter = wl.n_iter if n_iter is None else n_iter
    n_sweeps = wl.n_sweeps if n_sweeps is None else n_sweeps
    walkers = wl.walkers_per_system if walkers is None else walkers
    seed = wl.seed if seed is None else seed
    pos0 = workloads.initial_positions(wl)[sys_index]
    ws = [Walker(sysd, pos0, walker_offset + i, seed) for i in range(walkers)]
    W = Weights(sp.e_lo, wl.bin_width, sp.n_bins, beta_min=wl.beta_min, beta_max=wl.beta_max)
    mv = move_params(wl)
    out = dict(beta=[], alpha=[], g=[], hist=[], flat=[])
    for _ in range(n_iter):
        H = np.zeros(sp.n_bins, dtype=np.uint64)
        for w in ws:
            w.run(W, mv, n_sweeps, H)
        W.berg_update(H)
        out["beta"].append(W.beta.copy()); out["alpha"].append(W.alpha.copy())
        out["g"].append(W.g.copy()); out["hist"].append(H)
        out["flat"].append(flatness(H))
    res = {k: np.array(v) for k, v in out.items()}
    res["walkers"] = ws
    res["weights"] = W
    return res
