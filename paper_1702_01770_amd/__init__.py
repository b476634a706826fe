"""MI355X-native multicanonical (MUCA) sampler for coarse-grained AB heteropolymers.

Hot path of Frigori, "PHAST: Protein-like Heteropolymer Analysis by Statistical Thermodynamics"
(arXiv:1702.01770): MUCA Metropolis sweeps (Sec. 2.2, 3.2), Berg's weight recursion between
iterations (Sec. 2.2), the microcanonical analysis (Eqs. 4-8), plus an energy backward kernel
and canonical reweighting for force-field gradients.

Every step runs in the HIP library `libmuca.so` (C ABI in include/muca.h); this package only
marshals arguments.  It fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import MucaError, check, load

__all__ = ["Muca", "MucaError", "microcanonical_analyze", "reweight_fwd", "reweight_bwd",
           "load"]

PREC_FP64 = 0
PREC_FP32_SPLIT = 1


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class Muca:
    """One context: a batch of systems, each with `walkers_per_system` Markov chains that share
    the system's weights (parallel MUCA, Sec. 2.2 / Fig. 2)."""

    def __init__(self, chains_per_system: Sequence[int], chain_len: Sequence[int], types,
                 init_pos, c_lj, e_lo: Sequence[float], n_bins: Sequence[int], *,
                 walkers_per_system: int, k_lj_intra=4.0, k_lj_inter=4.0, k_bend=0.25,
                 k_tors=0.0, box_kind=0, box_len=0.0, bin_width=0.05, seed=1702,
                 precision=PREC_FP64, resync_sweeps=0, drift_tol=0.0, crank_max=np.pi / 3,
                 cap_rho=0.8, trans_max=0.3, rigid_per_sweep=0, pivot_per_sweep=0, pivot_max=0.5236,
                 rotate_per_sweep=0, rotate_max=0.5236, beta_min=0.0, beta_max=0.0,
                 waves_per_block=0, walkers_per_wave=0, stream: Optional[int] = None):
        L = load()
        self._keep = dict(
            cps=np.ascontiguousarray(chains_per_system, dtype=np.int32),
            cl=np.ascontiguousarray(chain_len, dtype=np.int32),
            ty=np.ascontiguousarray(types, dtype=np.uint8),
            pos=np.ascontiguousarray(init_pos, dtype=np.float64),
            c=np.ascontiguousarray(c_lj, dtype=np.float64),
            elo=np.ascontiguousarray(e_lo, dtype=np.float64),
            nb=np.ascontiguousarray(n_bins, dtype=np.int32))
        k = self._keep
        self.n_systems = len(k["cps"])
        self.walkers = int(walkers_per_system)
        off = np.concatenate([[0], np.cumsum(k["cps"])])
        self.n_beads = [int(k["cl"][off[s]:off[s + 1]].sum()) for s in range(self.n_systems)]
        self.n_bins = [int(x) for x in k["nb"]]
        self.e_lo = [float(x) for x in k["elo"]]
        self.bin_width = float(bin_width)
        cfg = _lib.MucaConfig(
            self.n_systems, int(k["c"].shape[0]), _ptr(k["cps"], C.c_int32),
            _ptr(k["cl"], C.c_int32), _ptr(k["ty"], C.c_uint8), _ptr(k["pos"], C.c_double),
            _ptr(k["c"], C.c_double), k_lj_intra, k_lj_inter, k_bend, k_tors, int(box_kind),
            float(box_len), _ptr(k["elo"], C.c_double), _ptr(k["nb"], C.c_int32),
            float(bin_width), self.walkers, int(seed), int(precision), int(resync_sweeps),
            float(drift_tol), float(crank_max), float(cap_rho), float(trans_max),
            int(rigid_per_sweep), int(pivot_per_sweep), float(pivot_max), int(rotate_per_sweep),
            float(rotate_max), float(beta_min), float(beta_max), int(waves_per_block),
            int(walkers_per_wave), stream)
        h = C.c_void_p()
        check(L.muca_init(C.byref(cfg), C.byref(h)))
        self._h = h
        self._L = L

    @classmethod
    def from_workload(cls, wl, init_pos, walkers: Optional[int] = None,
                      precision: Optional[int] = None, stream=None, systems=None, **over):
        """Build a context from a workload description (an object with the attributes of
        workloads.Workload) and the per-system starting coordinates init_pos[s] ([N_s, 3])."""
        import numpy as _np
        sel = list(range(len(wl.systems))) if systems is None else list(systems)
        syss = [wl.systems[i] for i in sel]
        pos = [init_pos[i] for i in sel]
        kw = dict(walkers_per_system=wl.walkers_per_system if walkers is None else walkers,
                  k_lj_intra=wl.k_lj_intra, k_lj_inter=wl.k_lj_inter, k_bend=wl.k_bend,
                  k_tors=wl.k_tors, box_kind=wl.box_kind, box_len=wl.box_len,
                  bin_width=wl.bin_width, seed=wl.seed,
                  precision=wl.precision if precision is None else precision,
                  resync_sweeps=wl.resync_sweeps, crank_max=wl.crank_max, cap_rho=wl.cap_rho,
                  trans_max=wl.trans_max, rigid_per_sweep=wl.rigid_per_sweep,
                  pivot_per_sweep=wl.pivot_per_sweep, pivot_max=wl.pivot_max,
                  rotate_per_sweep=wl.rotate_per_sweep, rotate_max=wl.rotate_max,
                  beta_min=getattr(wl, "beta_min", 0.0), beta_max=getattr(wl, "beta_max", 0.0),
                  stream=stream)
        kw.update(over)
        return cls([len(sp.chain_len) for sp in syss],
                   _np.concatenate([sp.chain_len for sp in syss]),
                   _np.concatenate([sp.types for sp in syss]),
                   _np.concatenate(pos), wl.c_lj, [sp.e_lo for sp in syss],
                   [sp.n_bins for sp in syss], **kw)

    # ---- lifecycle ----
    def close(self):
        if getattr(self, "_h", None):
            self._L.muca_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ck(self, rc):
        check(rc, self._h)

    # ---- sampling ----
    def sweep(self, n_sweeps: int):
        self._ck(self._L.muca_sweep(self._h, int(n_sweeps)))

    def hmc(self, n_traj: int, n_steps: int, step: float):
        """n_traj hybrid Monte Carlo trajectories of every walker (n_steps leapfrog steps of
        length step) under the current weights; one histogram count per trajectory."""
        self._ck(self._L.muca_hmc(self._h, int(n_traj), int(n_steps), float(step)))

    def update_weights(self):
        st = (_lib.IterStats * self.n_systems)()
        self._ck(self._L.muca_update_weights(self._h, st))
        return [dict(iteration=s.iteration, moves=s.moves, cvar=s.cvar, max_peak=s.max_peak,
                     k_min=s.k_min, k_max=s.k_max) for s in st]

    def iterate(self, n_sweeps: int, n_iter: int):
        self._ck(self._L.muca_iterate(self._h, int(n_sweeps), int(n_iter)))

    def stats_history(self, first: int, count: int):
        """[count, n_systems, 5]: moves, cvar, max_peak, k_min, k_max of iterations first.."""
        st = (_lib.IterStats * (self.n_systems * count))()
        self._ck(self._L.muca_get_stats_history(self._h, int(first), int(count), st))
        out = np.zeros((count, self.n_systems, 5))
        for i in range(count):
            for s in range(self.n_systems):
                x = st[i * self.n_systems + s]
                out[i, s] = (x.moves, x.cvar, x.max_peak, x.k_min, x.k_max)
        return out

    def synchronize(self):
        self._ck(self._L.muca_synchronize(self._h))

    def histogram(self, sys: int = 0, last: bool = False) -> np.ndarray:
        out = np.zeros(self.n_bins[sys], dtype=np.uint64)
        self._ck(self._L.muca_get_histogram(self._h, sys, int(last), _ptr(out, C.c_uint64),
                                            self.n_bins[sys]))
        return out

    def weights(self, sys: int = 0):
        K = self.n_bins[sys]
        b, a, g = np.zeros(K), np.zeros(K), np.zeros(K)
        self._ck(self._L.muca_get_weights(self._h, sys, _ptr(b, C.c_double), _ptr(a, C.c_double),
                                          _ptr(g, C.c_double), K))
        return b, a, g

    def set_weights(self, sys: int, beta, alpha, g=None):
        K = self.n_bins[sys]
        b = np.ascontiguousarray(beta, dtype=np.float64)
        a = np.ascontiguousarray(alpha, dtype=np.float64)
        gg = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
        self._ck(self._L.muca_set_weights(self._h, sys, _ptr(b, C.c_double), _ptr(a, C.c_double),
                                          None if gg is None else _ptr(gg, C.c_double), K))

    def walkers_state(self, sys: int = 0):
        """(pos [W, N, 3], energy [W], counters dict of arrays)."""
        W, N = self.walkers, self.n_beads[sys]
        pos = np.zeros((W, N, 3))
        e = np.zeros(W)
        cnt = (_lib.WalkerCounters * W)()
        self._ck(self._L.muca_get_walkers(self._h, sys, _ptr(pos, C.c_double), _ptr(e, C.c_double),
                                          cnt))
        fields = [f[0] for f in _lib.WalkerCounters._fields_]
        c = {f: np.array([getattr(x, f) for x in cnt]) for f in fields}
        return pos, e, c

    def set_walkers(self, sys: int, pos, sweeps=None):
        p = np.ascontiguousarray(pos, dtype=np.float64)
        sw = None if sweeps is None else np.ascontiguousarray(sweeps, dtype=np.uint64)
        self._ck(self._L.muca_set_walkers(self._h, sys, _ptr(p, C.c_double),
                                          None if sw is None else _ptr(sw, C.c_uint64)))

    def set_accept_log(self, n_moves: int):
        self._accept_moves = int(n_moves)
        self._ck(self._L.muca_set_accept_log(self._h, int(n_moves)))

    def accept_log(self, sys: int = 0) -> np.ndarray:
        out = np.zeros((self.walkers, self._accept_moves), dtype=np.uint8)
        self._ck(self._L.muca_get_accept_log(self._h, sys, _ptr(out, C.c_uint8),
                                             self._accept_moves))
        return out

    def get_state(self) -> bytes:
        n = C.c_size_t(0)
        self._ck(self._L.muca_get_state(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._ck(self._L.muca_get_state(self._h, buf, C.byref(n)))
        return buf.raw

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._ck(self._L.muca_set_state(self._h, buf, len(blob)))

    def autotune(self, probe_sweeps: int = 20) -> int:
        ch = C.c_int32(0)
        self._ck(self._L.muca_autotune(self._h, int(probe_sweeps), C.byref(ch)))
        return ch.value

    def launch_info(self) -> dict:
        """Current sweep launch plan (walkers per wave, waves per block, pairing, workgroups,
        LDS bytes, sweeps per launch)."""
        li = _lib.LaunchInfo()
        self._ck(self._L.muca_get_launch_info(self._h, C.byref(li)))
        return {f: getattr(li, f) for f, _ in li._fields_}

    # ---- differentiation (device pointers, e.g. torch tensors' data_ptr()) ----
    def energy_fwd_ptr(self, sys: int, x_ptr: int, n_cfg: int, theta, e_ptr: int):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        self._ck(self._L.muca_energy_fwd(self._h, sys, C.c_void_p(x_ptr), int(n_cfg),
                                         _ptr(th, C.c_double), C.c_void_p(e_ptr)))

    def energy_bwd_ptr(self, sys: int, x_ptr: int, n_cfg: int, theta, ge_ptr: int, gx_ptr: int,
                       gth_ptr: int):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        self._ck(self._L.muca_energy_bwd(self._h, sys, C.c_void_p(x_ptr), int(n_cfg),
                                         _ptr(th, C.c_double), C.c_void_p(ge_ptr),
                                         C.c_void_p(gx_ptr), C.c_void_p(gth_ptr)))


def reweight_workspace_bytes(n: int, n_t: int) -> int:
    return int(load().muca_reweight_workspace_bytes(int(n), int(n_t)))


def reweight_fwd(e_ptr, lnw0_ptr, n, temps, mean_ptr, cv_ptr, mom_ptr, ws_ptr, ws_bytes, stream):
    t = np.ascontiguousarray(temps, dtype=np.float64)
    check(load().muca_reweight_fwd(C.c_void_p(e_ptr), C.c_void_p(lnw0_ptr), int(n),
                                   _ptr(t, C.c_double), len(t), C.c_void_p(mean_ptr),
                                   C.c_void_p(cv_ptr), C.c_void_p(mom_ptr), C.c_void_p(ws_ptr),
                                   int(ws_bytes), C.c_void_p(stream)))


def reweight_fwd_noalloc(e_ptr, lnw0_ptr, n, temps, mean_ptr, cv_ptr, mom_ptr, stream):
    """muca_reweight_fwd with the library's static per-GPU workspace (no allocation)."""
    t = np.ascontiguousarray(temps, dtype=np.float64)
    check(load().muca_reweight_fwd_noalloc(C.c_void_p(e_ptr), C.c_void_p(lnw0_ptr), int(n),
                                           _ptr(t, C.c_double), len(t), C.c_void_p(mean_ptr),
                                           C.c_void_p(cv_ptr), C.c_void_p(mom_ptr),
                                           C.c_void_p(stream)))


def reweight_bwd(e_ptr, lnw0_ptr, n, temps, mom_ptr, gmean_ptr, gcv_ptr, ge_ptr, stream):
    t = np.ascontiguousarray(temps, dtype=np.float64)
    check(load().muca_reweight_bwd(C.c_void_p(e_ptr), C.c_void_p(lnw0_ptr), int(n),
                                   _ptr(t, C.c_double), len(t), C.c_void_p(mom_ptr),
                                   C.c_void_p(gmean_ptr), C.c_void_p(gcv_ptr), C.c_void_p(ge_ptr),
                                   C.c_void_p(stream)))


def microcanonical_analyze(beta_hist, alpha_hist, e_lo, bin_width, k_lo, k_hi, n_s, n_e, block,
                           dE, beta_c=0.0, tol_beta=0.0, tol_l=0.0, n_monomers=1) -> dict:
    """Microcanonical analysis (Eqs. 4-8) of iterations [n_s, n_e) on bins [k_lo, k_hi)."""
    B = np.ascontiguousarray(beta_hist, dtype=np.float64)
    A = np.ascontiguousarray(alpha_hist, dtype=np.float64)
    n_iter, K = B.shape
    G = int(k_hi - k_lo)
    arrs = {k: np.zeros(G) for k in ("E", "S", "dS", "beta", "dbeta", "cv", "dcv", "F", "dF")}
    ain = _lib.AnalysisIn(_ptr(B, C.c_double), _ptr(A, C.c_double), n_iter, K, float(e_lo),
                          float(bin_width), int(k_lo), int(k_hi), int(n_s), int(n_e), int(block),
                          float(dE), float(beta_c), float(tol_beta), float(tol_l), int(n_monomers))
    aout = _lib.AnalysisOut()
    aout.n_grid = G
    for k, v in arrs.items():
        setattr(aout, k, _ptr(v, C.c_double))
    check(load().microcanonical_analyze(C.byref(ain), C.byref(aout)))
    res = dict(arrs)
    for k in ("beta_c", "dbeta_c", "latent", "dlatent", "barrier", "dbarrier", "n_blocks"):
        res[k] = getattr(aout, k)
    return res
