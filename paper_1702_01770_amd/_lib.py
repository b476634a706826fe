"""ctypes declarations of the C ABI in include/muca.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmuca.so")

MUCA_OK = 0
ERRORS = {-1: "MUCA_E_INVAL", -2: "MUCA_E_NOMEM", -3: "MUCA_E_DEVICE", -4: "MUCA_E_WINDOW",
          -5: "MUCA_E_DRIFT", -6: "MUCA_E_STATE"}


class MucaConfig(C.Structure):
    _fields_ = [("n_systems", C.c_int32), ("n_types", C.c_int32),
                ("chains_per_system", C.POINTER(C.c_int32)), ("chain_len", C.POINTER(C.c_int32)),
                ("types", C.POINTER(C.c_uint8)), ("init_pos", C.POINTER(C.c_double)),
                ("c_lj", C.POINTER(C.c_double)),
                ("k_lj_intra", C.c_double), ("k_lj_inter", C.c_double), ("k_bend", C.c_double),
                ("k_tors", C.c_double), ("box_kind", C.c_int32), ("box_len", C.c_double),
                ("e_lo", C.POINTER(C.c_double)), ("n_bins", C.POINTER(C.c_int32)),
                ("bin_width", C.c_double), ("walkers_per_system", C.c_int32),
                ("seed", C.c_uint64), ("precision", C.c_int32), ("resync_sweeps", C.c_int32),
                ("drift_tol", C.c_double), ("crank_max", C.c_double), ("cap_rho", C.c_double),
                ("trans_max", C.c_double), ("rigid_per_sweep", C.c_int32),
                ("pivot_per_sweep", C.c_int32), ("pivot_max", C.c_double),
                ("rotate_per_sweep", C.c_int32), ("rotate_max", C.c_double),
                ("beta_min", C.c_double), ("beta_max", C.c_double),
                ("waves_per_block", C.c_int32), ("walkers_per_wave", C.c_int32),
                ("stream", C.c_void_p)]


class IterStats(C.Structure):
    _fields_ = [("iteration", C.c_int64), ("moves", C.c_int64), ("cvar", C.c_double),
                ("max_peak", C.c_double), ("k_min", C.c_int32), ("k_max", C.c_int32)]


class WalkerCounters(C.Structure):
    _fields_ = [("moves", C.c_uint64), ("accepted", C.c_uint64), ("rigid_moves", C.c_uint64),
                ("rigid_accepted", C.c_uint64), ("window_rejects", C.c_uint64),
                ("sweeps", C.c_uint64), ("max_drift", C.c_double),
                ("pivot_moves", C.c_uint64), ("pivot_accepted", C.c_uint64),
                ("rot_moves", C.c_uint64), ("rot_accepted", C.c_uint64),
                ("hmc_trajectories", C.c_uint64), ("hmc_accepted", C.c_uint64)]


class LaunchInfo(C.Structure):
    _fields_ = [("walkers_per_wave", C.c_int32), ("waves_per_block", C.c_int32),
                ("paired", C.c_int32), ("workgroups", C.c_int32), ("lds_bytes", C.c_int64),
                ("sweeps_per_launch", C.c_int64), ("lanes_used", C.c_int32)]


class AnalysisIn(C.Structure):
    _fields_ = [("beta", C.POINTER(C.c_double)), ("alpha", C.POINTER(C.c_double)),
                ("n_iter", C.c_int32), ("n_bins", C.c_int32), ("e_lo", C.c_double),
                ("bin_width", C.c_double), ("k_lo", C.c_int32), ("k_hi", C.c_int32),
                ("n_s", C.c_int32), ("n_e", C.c_int32), ("block", C.c_int32), ("dE", C.c_double),
                ("beta_c", C.c_double), ("tol_beta", C.c_double), ("tol_l", C.c_double),
                ("n_monomers", C.c_int32)]


_DP = C.POINTER(C.c_double)


class AnalysisOut(C.Structure):
    _fields_ = [("n_grid", C.c_int32), ("E", _DP), ("S", _DP), ("dS", _DP), ("beta", _DP),
                ("dbeta", _DP), ("cv", _DP), ("dcv", _DP), ("F", _DP), ("dF", _DP),
                ("beta_c", C.c_double), ("dbeta_c", C.c_double), ("latent", C.c_double),
                ("dlatent", C.c_double), ("barrier", C.c_double), ("dbarrier", C.c_double),
                ("n_blocks", C.c_int32)]


EXPORTS = ["muca_init", "muca_sweep", "muca_hmc", "muca_update_weights", "muca_iterate",
           "muca_get_stats_history", "muca_synchronize", "muca_get_histogram",
           "muca_get_weights", "muca_set_weights", "muca_get_walkers", "muca_set_walkers",
           "muca_set_accept_log", "muca_get_accept_log", "muca_get_state", "muca_set_state",
           "muca_get_launch_info",
           "muca_autotune", "muca_energy_fwd", "muca_energy_bwd",
           "muca_reweight_workspace_bytes", "muca_reweight_fwd", "muca_reweight_fwd_noalloc",
           "muca_reweight_bwd",
           "microcanonical_analyze", "muca_last_error", "muca_destroy"]

_lib = None


def load():
    """Load libmuca.so (built by paper_1702_01770_amd.build); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() or "
                           "python paper_1702_01770_amd/build.py")
    try:
        # torch ships its own HIP runtime under the same soname; loading it first makes the
        # library bind to that single runtime, so torch streams and allocations are shared
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.muca_init.argtypes = [C.POINTER(MucaConfig), C.POINTER(vp)]
    L.muca_sweep.argtypes = [vp, i64]
    L.muca_hmc.argtypes = [vp, i64, i32, C.c_double]
    L.muca_update_weights.argtypes = [vp, C.POINTER(IterStats)]
    L.muca_iterate.argtypes = [vp, i64, i32]
    L.muca_get_stats_history.argtypes = [vp, i64, i32, C.POINTER(IterStats)]
    L.muca_synchronize.argtypes = [vp]
    L.muca_get_histogram.argtypes = [vp, i32, i32, C.POINTER(C.c_uint64), i32]
    L.muca_get_weights.argtypes = [vp, i32, _DP, _DP, _DP, i32]
    L.muca_set_weights.argtypes = [vp, i32, _DP, _DP, _DP, i32]
    L.muca_get_walkers.argtypes = [vp, i32, _DP, _DP, C.POINTER(WalkerCounters)]
    L.muca_set_walkers.argtypes = [vp, i32, _DP, C.POINTER(C.c_uint64)]
    L.muca_set_accept_log.argtypes = [vp, i64]
    L.muca_get_accept_log.argtypes = [vp, i32, C.POINTER(C.c_uint8), i64]
    L.muca_get_state.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
    L.muca_set_state.argtypes = [vp, vp, C.c_size_t]
    L.muca_autotune.argtypes = [vp, i64, C.POINTER(i32)]
    L.muca_energy_fwd.argtypes = [vp, i32, vp, i64, _DP, vp]
    L.muca_energy_bwd.argtypes = [vp, i32, vp, i64, _DP, vp, vp, vp]
    L.muca_reweight_workspace_bytes.restype = C.c_size_t
    L.muca_reweight_workspace_bytes.argtypes = [i64, i32]
    L.muca_reweight_fwd.argtypes = [vp, vp, i64, _DP, i32, vp, vp, vp, vp, C.c_size_t, vp]
    L.muca_reweight_fwd_noalloc.argtypes = [vp, vp, i64, _DP, i32, vp, vp, vp, vp]
    L.muca_reweight_bwd.argtypes = [vp, vp, i64, _DP, i32, vp, vp, vp, vp, vp]
    L.microcanonical_analyze.argtypes = [C.POINTER(AnalysisIn), C.POINTER(AnalysisOut)]
    L.muca_last_error.restype = C.c_char_p
    L.muca_last_error.argtypes = [vp]
    L.muca_destroy.argtypes = [vp]
    for name in EXPORTS:
        getattr(L, name).restype = getattr(L, name).restype if name in (
            "muca_reweight_workspace_bytes", "muca_last_error") else (
            None if name == "muca_destroy" else C.c_int)
    _lib = L
    return L


class MucaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def check(rc, ctx=None):
    if rc != MUCA_OK:
        msg = load().muca_last_error(ctx)
        raise MucaError(rc, msg.decode() if msg else "")
