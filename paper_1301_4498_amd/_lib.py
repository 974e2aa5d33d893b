"""ctypes binding of libnyxhydro.so (include/nyx_hydro.h): argument marshalling
only.  Every step of the path runs in the HIP library; if the library is not
built this module raises instead of falling back to anything."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnyxhydro.so")

NYX_OK = 0
NYX_FP64 = 0
NYX_MIXED = 1
NYX_RIEMANN_TWOSHOCK = 0
NYX_RIEMANN_LEARNED = 1
NYX_RIEMANN_LINEARIZED = 2
NYX_RECON_PPM = 0
NYX_RECON_PLM = 1
NYX_LAUNCH_STAGED = 0
NYX_LAUNCH_PERSISTENT = 1
NYX_LAUNCH_FUSED = 2

STATUS = {0: "NYX_OK", -1: "NYX_E_NULL", -2: "NYX_E_SHAPE", -3: "NYX_E_PARAM",
          -4: "NYX_E_ALIAS", -5: "NYX_E_HIP", -6: "NYX_E_UNSUPPORTED", -7: "NYX_E_WORKSPACE",
          -8: "NYX_E_SCRATCH"}


class Params(ctypes.Structure):
    _fields_ = [
        ("gamma", ctypes.c_double),
        ("eta_dual", ctypes.c_double),
        ("small_dens", ctypes.c_double),
        ("small_pres", ctypes.c_double),
        ("riemann_tol", ctypes.c_double),
        ("mlp_resid_tol", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("riemann_maxiter", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("riemann", ctypes.c_int32),
        ("learned_stages_mask", ctypes.c_int32),
        ("recon", ctypes.c_int32),
        ("grav_energy_form", ctypes.c_int32),
        ("mlp_weights", ctypes.c_void_p),
        ("mixed_riemann_stop", ctypes.c_double),
    ]


class Box(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("ng", ctypes.c_int32),
        ("state_off", ctypes.c_int64),
        ("grav_off", ctypes.c_int64),
        ("comp_stride", ctypes.c_int64),
        ("grav_stride", ctypes.c_int64),
        ("dx", ctypes.c_double),
    ]


STATS_FIELDS = ("nonfinite", "neg_dens", "neg_eint", "floor_hits", "trans_reverts",
                "sync_E_from_e", "riemann_iters", "riemann_calls", "mlp_used", "mlp_fallback")


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_ulonglong) for n in STATS_FIELDS]


class NyxError(RuntimeError):
    def __init__(self, fn, rc):
        super().__init__("%s failed: %s (%d)" % (fn, STATUS.get(rc, "?"), rc))
        self.rc = rc


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libnyxhydro.so is not built (run __graft_entry__.build() or "
                               "python paper_1301_4498_amd/build.py); there is no fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        P, B = ctypes.POINTER(Params), ctypes.POINTER(Box)
        d, i = ctypes.c_double, ctypes.c_int
        sig = {
            "nyx_default_params": (None, [P]),
            "nyx_status_string": (ctypes.c_char_p, [i]),
            "nyx_workspace_bytes": (i, [P, B, ctypes.POINTER(sz)]),
            "nyx_estimate_dt": (i, [P, B, vp, d, d, vp, vp, sz, vp]),
            "nyx_hydro_step": (i, [P, B, vp, vp, d, d, d, vp, vp, vp, vp, sz, vp]),
            "nyx_hydro_step_noalloc": (i, [P, B, vp, vp, d, d, d, vp, vp, vp, vp]),
            "nyx_noalloc_max_bytes": (i, [ctypes.POINTER(sz)]),
            "nyx_batch_workspace_bytes": (i, [P, i, B, ctypes.POINTER(sz), ctypes.POINTER(sz)]),
            "nyx_batch_create": (i, [P, i, B, vp, sz, vp, ctypes.POINTER(vp)]),
            "nyx_batch_destroy": (i, [vp]),
            "nyx_batch_num_groups": (i, [vp]),
            "nyx_batch_estimate_dt": (i, [vp, vp, d, d, vp, vp]),
            "nyx_batch_min_dt": (i, [vp, vp, vp]),
            "nyx_hydro_step_batched": (i, [vp, vp, vp, vp, d, d, vp, vp, vp, vp]),
            "nyx_fill_ghosts_periodic": (i, [B, vp, i, vp]),
            "nyx_batch_fill_ghosts": (i, [vp, i, i, i, i, vp, vp]),
            "nyx_batch_set_ghost_source": (i, [vp, i, i, i, i]),
            "nyx_profile_enable": (i, [i]),
            "nyx_batch_set_harvest": (i, [vp, vp, vp, ctypes.c_longlong, d, ctypes.c_ulonglong]),
            "nyx_mlp_init": (i, [vp, ctypes.c_ulonglong, vp]),
            "nyx_mlp_loss_grad": (i, [vp, vp, ctypes.c_longlong, d, d, vp, vp, vp]),
            "nyx_mlp_adam": (i, [vp, vp, vp, vp, i, d, d, d, d, vp]),
            "nyx_mlp_pack": (i, [vp, vp, vp]),
            "nyx_mlp_predict": (i, [vp, vp, ctypes.c_longlong, d, vp, vp]),
            "nyx_profile_read": (i, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong), i]),
            "nyx_batch_autotune": (i, [vp, vp, vp, vp, d, d, vp, vp, i, ctypes.POINTER(ctypes.c_float),
                                       ctypes.POINTER(i), vp]),
            "nyx_batch_set_tuning": (i, [vp, ctypes.POINTER(i)]),
            "nyx_batch_set_launch_mode": (i, [vp, i]),
            "nyx_batch_get_launch_mode": (i, [vp, ctypes.POINTER(i)]),
            "nyx_batch_persistent_aborted": (i, [vp, ctypes.POINTER(i), vp]),
            "nyx_batch_autotune_mode": (i, [vp, vp, vp, vp, d, d, vp, i, ctypes.POINTER(ctypes.c_float),
                                            ctypes.POINTER(i), vp]),
            "nyx_fill_plan_bytes": (i, [i, B, ctypes.POINTER(i), ctypes.POINTER(i), i, B,
                                        ctypes.POINTER(i), ctypes.POINTER(sz)]),
            "nyx_fill_plan_create": (i, [i, B, ctypes.POINTER(i), ctypes.POINTER(i), i, B,
                                         ctypes.POINTER(i), vp, sz, vp, ctypes.POINTER(vp)]),
            "nyx_fill_plan_counts": (i, [vp, ctypes.POINTER(ctypes.c_longlong),
                                         ctypes.POINTER(ctypes.c_longlong)]),
            "nyx_fill_level": (i, [vp, vp, vp, i, vp]),
            "nyx_fill_level_time": (i, [vp, vp, vp, vp, d, i, vp]),
            "nyx_fill_plan_destroy": (i, [vp]),
            "nyx_batch_get_tuning": (i, [vp, ctypes.POINTER(i)]),
            "nyx_sync_plan_bytes": (i, [i, B, ctypes.POINTER(i), ctypes.POINTER(i), i, B,
                                        ctypes.POINTER(i), ctypes.POINTER(sz)]),
            "nyx_sync_plan_create": (i, [i, B, ctypes.POINTER(i), ctypes.POINTER(i), i, B,
                                         ctypes.POINTER(i), vp, sz, vp, ctypes.POINTER(vp)]),
            "nyx_sync_plan_counts": (i, [vp, ctypes.POINTER(ctypes.c_longlong),
                                         ctypes.POINTER(ctypes.c_longlong),
                                         ctypes.POINTER(ctypes.c_longlong)]),
            "nyx_sync_plan_destroy": (i, [vp]),
            "nyx_batch_set_flux_register": (i, [vp, vp, i, vp]),
            "nyx_reflux": (i, [vp, vp, vp, i, vp]),
            "nyx_average_down": (i, [vp, vp, vp, i, vp]),
            "nyx_cic_deposit": (i, [vp, vp, ctypes.c_longlong, ctypes.POINTER(i), d, vp, vp]),
            "nyx_poisson_workspace_bytes": (i, [ctypes.POINTER(i), ctypes.POINTER(sz)]),
            "nyx_poisson_solve": (i, [ctypes.POINTER(i), d, d, vp, vp, ctypes.POINTER(Box), vp, d,
                                      i, vp, sz, vp, ctypes.POINTER(i),
                                      ctypes.POINTER(ctypes.c_double)]),
            "nyx_gravity_from_phi": (i, [ctypes.POINTER(i), d, vp, ctypes.POINTER(Box), vp, i,
                                         vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(fn: str, rc: int) -> None:
    if rc != NYX_OK:
        raise NyxError(fn, rc)


def exported_symbols():
    return ["nyx_default_params", "nyx_status_string", "nyx_workspace_bytes", "nyx_estimate_dt",
            "nyx_hydro_step", "nyx_batch_workspace_bytes", "nyx_batch_create",
            "nyx_batch_destroy", "nyx_batch_num_groups", "nyx_batch_estimate_dt",
            "nyx_batch_min_dt", "nyx_hydro_step_batched", "nyx_fill_ghosts_periodic",
            "nyx_batch_fill_ghosts", "nyx_batch_set_ghost_source", "nyx_profile_enable",
            "nyx_profile_read",
            "nyx_batch_set_harvest", "nyx_mlp_init", "nyx_mlp_loss_grad", "nyx_mlp_adam",
            "nyx_mlp_pack", "nyx_mlp_predict", "nyx_batch_autotune", "nyx_batch_set_tuning",
            "nyx_batch_get_tuning", "nyx_fill_plan_bytes", "nyx_fill_plan_create",
            "nyx_fill_plan_counts", "nyx_fill_level", "nyx_fill_level_time", "nyx_fill_plan_destroy",
            "nyx_sync_plan_bytes", "nyx_sync_plan_create", "nyx_sync_plan_counts",
            "nyx_sync_plan_destroy", "nyx_batch_set_flux_register", "nyx_reflux",
            "nyx_average_down", "nyx_cic_deposit", "nyx_poisson_workspace_bytes",
            "nyx_poisson_solve", "nyx_gravity_from_phi", "nyx_hydro_step_noalloc",
            "nyx_noalloc_max_bytes", "nyx_batch_set_launch_mode", "nyx_batch_get_launch_mode",
            "nyx_batch_persistent_aborted", "nyx_batch_autotune_mode"]

TUNE_CANDIDATES = 16
MLP_NPARAM = 9349
MLP_PACKED_BYTES = 23552


STAGE_NAMES = ("prim", "flat", "trace", "riem0", "riem1", "riem2", "update")
STAGES = len(STAGE_NAMES)


def profile_enable(on: bool) -> None:
    check("nyx_profile_enable", lib().nyx_profile_enable(1 if on else 0))


def profile_read(reset: bool = True):
    """Milliseconds accumulated per stage and the number of timed sequences."""
    ms = (ctypes.c_double * len(STAGE_NAMES))()
    n = ctypes.c_longlong(0)
    check("nyx_profile_read", lib().nyx_profile_read(ms, ctypes.byref(n), 1 if reset else 0))
    return dict(zip(STAGE_NAMES, list(ms))), n.value
