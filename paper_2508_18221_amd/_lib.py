"""ctypes binding of libgrmhd.so (argument marshalling only).

Every computation runs in the HIP library; this module only describes the
C-ABI of include/grmhd.h to Python.  Loading fails loudly when the library has
not been built (python -m paper_2508_18221_amd.build)."""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# GRMHD_LIBRARY selects another build of the library (the host-sanitizer
# build of the CPU tests); the default is the in-tree libgrmhd.so
LIB_PATH = os.environ.get("GRMHD_LIBRARY") or os.path.join(HERE, "libgrmhd.so")

GRMHD_FP64, GRMHD_MIX_FP32, GRMHD_MIX_BF16X3, GRMHD_STORE_FP32 = 0, 1, 2, 3
NFIELDS = 32


class Grid(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("nth", ctypes.c_int32), ("nph", ctypes.c_int32),
                ("r_in", ctypes.c_double), ("r_out", ctypes.c_double),
                ("th_min", ctypes.c_double), ("th_max", ctypes.c_double),
                ("filt_alpha", ctypes.c_double), ("filt_order", ctypes.c_int32),
                ("filter_on", ctypes.c_int32), ("dealias", ctypes.c_int32)]


class Phys(ctypes.Structure):
    _fields_ = [("M", ctypes.c_double), ("a", ctypes.c_double), ("gamma_ad", ctypes.c_double),
                ("cfl", ctypes.c_double), ("eta", ctypes.c_double),
                ("cowling", ctypes.c_int32), ("gauge_k0", ctypes.c_int32),
                ("r_c", ctypes.c_double), ("rho_c", ctypes.c_double), ("beta_min", ctypes.c_double),
                ("pert_amp", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("rho_floor", ctypes.c_double), ("p_floor", ctypes.c_double),
                ("id_kind", ctypes.c_int32), ("tor_r_in", ctypes.c_double), ("tor_r_max", ctypes.c_double),
                ("tor_rho_max", ctypes.c_double), ("tor_atm", ctypes.c_double), ("tor_loop_cut", ctypes.c_double),
                ("glm", ctypes.c_int32), ("glm_ch", ctypes.c_double), ("glm_tau", ctypes.c_double),
                ("split", ctypes.c_int32), ("c2p_damped", ctypes.c_int32)]


class Diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("step", ctypes.c_int64), ("c2p_fail", ctypes.c_int64),
                ("nonfinite", ctypes.c_int64), ("rest_mass", ctypes.c_double),
                ("entropy", ctypes.c_double), ("max_abs_divB", ctypes.c_double),
                ("min_alpha", ctypes.c_double), ("max_W", ctypes.c_double),
                ("ham_l2", ctypes.c_double), ("ham_linf", ctypes.c_double),
                ("mom_l2", ctypes.c_double), ("mom_linf", ctypes.c_double)]


class JobInfo(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("state", ctypes.c_int32), ("nr", ctypes.c_int32),
                ("nth", ctypes.c_int32), ("nph", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("steps_done", ctypes.c_int64), ("steps_total", ctypes.c_int64), ("dt", ctypes.c_double),
                ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("latency", ctypes.c_double), ("bytes", ctypes.c_size_t)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("running", ctypes.c_int64), ("queued", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("p50_latency", ctypes.c_double),
                ("p99_latency", ctypes.c_double), ("mean_latency", ctypes.c_double),
                ("point_stage_updates", ctypes.c_double), ("wall", ctypes.c_double), ("busy", ctypes.c_double),
                ("bytes_in_use", ctypes.c_size_t), ("bytes_peak", ctypes.c_size_t)]


_P = ctypes.POINTER
_dp = _P(ctypes.c_double)
_vp = ctypes.c_void_p

# name -> (restype, argtypes); the same names as include/grmhd.h
SIGNATURES = {
    "grmhd_query_bytes": (ctypes.c_int, [_P(Grid), ctypes.c_int, _P(ctypes.c_size_t), _P(ctypes.c_size_t)]),
    "grmhd_create": (ctypes.c_int, [_P(Grid), _P(Phys), ctypes.c_int, _vp, _vp, _vp, _P(_vp)]),
    "grmhd_destroy": (ctypes.c_int, [_vp]),
    "grmhd_init_state": (ctypes.c_int, [_vp]),
    "grmhd_set_state": (ctypes.c_int, [_vp, _dp, ctypes.c_size_t, _dp, ctypes.c_double]),
    "grmhd_get_state": (ctypes.c_int, [_vp, _dp, ctypes.c_size_t, _dp]),
    "grmhd_state_ptr": (ctypes.c_int, [_vp, _P(_vp), _P(_vp)]),
    "grmhd_rhs": (ctypes.c_int, [_vp, _vp, _vp]),
    "grmhd_step": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "grmhd_step_noalloc": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "grmhd_diagnostics": (ctypes.c_int, [_vp, _P(Diag)]),
    "grmhd_dt": (ctypes.c_double, [_vp]),
    "grmhd_time": (ctypes.c_double, [_vp]),
    "grmhd_last_error": (ctypes.c_char_p, []),
    "grmhd_apply_operator": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, ctypes.c_int32]),
    "grmhd_con2prim": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "grmhd_xcts_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "grmhd_profile_step": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, ctypes.c_int32, _P(ctypes.c_int32)]),
    "grmhd_step_batch": (ctypes.c_int, [_P(_vp), ctypes.c_int32, ctypes.c_int32]),
    "grmhd_set_dt": (ctypes.c_int, [_vp, ctypes.c_double]),
    "grmhd_set_stream": (ctypes.c_int, [_vp, _vp]),
    "grmhd_time_step": (ctypes.c_int, [_P(Grid), ctypes.c_double, _dp]),
    "grmhd_server_create": (ctypes.c_int, [_vp, ctypes.c_size_t, ctypes.c_int32, _vp, _P(_vp)]),
    "grmhd_server_destroy": (ctypes.c_int, [_vp]),
    "grmhd_server_submit": (ctypes.c_int, [_vp, _P(Grid), _P(Phys), ctypes.c_int, ctypes.c_double,
                                           ctypes.c_int32, _P(ctypes.c_int64)]),
    "grmhd_server_tick": (ctypes.c_int, [_vp, _P(ctypes.c_int32)]),
    "grmhd_server_poll": (ctypes.c_int, [_vp, ctypes.c_int64, _P(JobInfo)]),
    "grmhd_server_cancel": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "grmhd_server_result": (ctypes.c_int, [_vp, ctypes.c_int64, _dp, ctypes.c_size_t]),
    "grmhd_server_stats": (ctypes.c_int, [_vp, _P(ServerStats)]),
    "grmhd_server_clock": (ctypes.c_double, [_vp]),
    "grmhd_server_last_error": (ctypes.c_char_p, []),
}

KERNEL_KINDS = ["c2p_flux", "deriv_r2", "deriv_r1", "deriv_t2", "deriv_t1", "deriv_p2", "deriv_p1",
                "rhs_rk", "filter_r", "filter_t", "filter_p", "deriv_r", "deriv_t", "deriv_p", "ricci",
                "dflux_r", "dflux_t", "dflux_p"]

_lib = None


def load():
    """Load libgrmhd.so (once) and attach the prototypes."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2508_18221_amd.build`")
    # PyTorch wheels ship their own HIP runtime.  Device memory and streams
    # handed to the library come from that runtime, so the library must bind
    # to the same copy: load torch first, and the dynamic loader resolves
    # libamdhip64.so.7 to the already-loaded runtime instead of a second one.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class GrmhdError(RuntimeError):
    pass


def check(rc):
    if rc != 0:
        msg = load().grmhd_last_error().decode(errors="replace")
        raise GrmhdError(f"grmhd error {rc}: {msg}")
    return rc


def check_server(rc):
    if rc != 0:
        msg = load().grmhd_server_last_error().decode(errors="replace")
        raise GrmhdError(f"grmhd server error {rc}: {msg}")
    return rc
