"""ctypes declarations of the C ABI in include/msd_afqmc.h (no computation here)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MSD_AFQMC_LIB", os.path.join(_HERE, "libmsd_afqmc.so"))

MSD_OK = 0
STATUS = {
    0: "MSD_OK", -1: "MSD_ERR_ARG", -2: "MSD_ERR_SHAPE", -3: "MSD_ERR_TRIAL",
    -4: "MSD_ERR_SINGULAR", -5: "MSD_ERR_DEVICE", -6: "MSD_ERR_OOM", -7: "MSD_ERR_STATE",
    -8: "MSD_ERR_UNSUPPORTED",
}


class MsdDims(C.Structure):
    _fields_ = [("M", C.c_int32), ("n_alpha", C.c_int32), ("n_beta", C.c_int32),
                ("n_chol", C.c_int32), ("n_walkers", C.c_int32), ("reserved", C.c_int32),
                ("n_det", C.c_int64)]


class MsdTuning(C.Structure):
    _fields_ = [("fb_splitk", C.c_int32), ("lambda_variant", C.c_int32),
                ("lambda_chunk", C.c_int32), ("second_gsplit", C.c_int32),
                ("second_stage", C.c_int32), ("second_gather", C.c_int32),
                ("second_copy", C.c_int32), ("second_waves", C.c_int32),
                ("walker_tile", C.c_int32), ("energy_form", C.c_int32),
                ("second_whole", C.c_int32), ("reserved", C.c_int32)]


class MsdOptions(C.Structure):
    _fields_ = [("n_taylor", C.c_int32), ("stabilize_freq", C.c_int32), ("timing", C.c_int32),
                ("energy_algo", C.c_int32), ("graphs", C.c_int32), ("precision", C.c_int32),
                ("mixed_tmax", C.c_double)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_vp = C.c_void_p

# name -> (restype, argtypes)
SIGNATURES = {
    "msd_status_string": (C.c_char_p, [C.c_int]),
    "msd_last_error": (C.c_char_p, [_vp]),
    "msd_default_options": (C.c_int, [C.POINTER(MsdOptions)]),
    "msd_create": (C.c_int, [C.POINTER(MsdDims), C.POINTER(MsdOptions), C.c_int32, _vp,
                             C.POINTER(_vp)]),
    "msd_destroy": (None, [_vp]),
    "msd_set_hamiltonian": (C.c_int, [_vp, _vp, _vp, C.c_double]),
    "msd_set_trial_occ": (C.c_int, [_vp, _vp, _vp, _vp]),
    "msd_set_trial_exc": (C.c_int, [_vp, _vp, _vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "msd_set_walkers": (C.c_int, [_vp, _vp, _vp, _vp]),
    "msd_set_walkers_dev": (C.c_int, [_vp, _vp, _vp, _vp]),
    "msd_get_walkers": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "msd_get_weights": (C.c_int, [_vp, _vp, _vp]),
    "msd_measure": (C.c_int, [_vp, C.c_double, _vp, _vp, _vp]),
    "msd_measure_dev": (C.c_int, [_vp, C.c_double, _vp, _vp, _vp]),
    "msd_propagate": (C.c_int, [_vp, _vp, C.c_double, C.c_double, C.c_int32]),
    "msd_propagate_dev": (C.c_int, [_vp, _vp, C.c_double, C.c_double, C.c_int32]),
    "msd_population_control": (C.c_int, [_vp, C.c_double, _vp]),
    "msd_population_control_dev": (C.c_int, [_vp, C.c_double, _vp]),
    "msd_population_control_noalloc": (C.c_int, [_vp, C.c_double, _vp]),
    "msd_run_block": (C.c_int, [_vp, _vp, C.c_double, C.c_double, C.c_int32, C.c_int32, _vp,
                                _vp]),
    "msd_get_green": (C.c_int, [_vp, C.c_int32, _vp, _vp]),
    "msd_get_timings": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_char_p), _dp,
                                  C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "msd_reset_timings": (C.c_int, [_vp]),
    "msd_get_measurement": (C.c_int, [_vp, _vp, _vp, _vp]),
    "msd_get_tuning": (C.c_int, [_vp, C.POINTER(MsdTuning)]),
    "msd_set_tuning": (C.c_int, [_vp, C.POINTER(MsdTuning)]),
    "msd_autotune": (C.c_int, [_vp, C.c_double, C.c_int32, C.POINTER(MsdTuning)]),
    "msd_batch_create": (C.c_int, [C.POINTER(_vp), C.c_int32, _vp, C.POINTER(_vp)]),
    "msd_batch_destroy": (None, [_vp]),
    "msd_batch_step": (C.c_int, [_vp, C.POINTER(_vp), C.c_double, C.c_double, C.c_int32]),
    "msd_trial_analyze": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int64, _vp, _vp, _vp,
                                    _vp, _vp]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises ImportError (never falls back) if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"libmsd_afqmc.so not found at {path}; build it with "
            "`python -m paper_2406_08314_amd.build` (there is no CPU fallback)")
    # One HIP runtime per process: PyTorch ships its own copy of the HIP
    # runtime (same soname).  Loading it first makes this library bind to it,
    # so device pointers and streams from torch are valid here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
