"""ctypes declarations mirroring include/stfdfd.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstfdfd.so")

STF_OK, STF_EINVAL, STF_ENOMEM, STF_EDEVICE, STF_ESTATE, STF_EPIVOT, STF_ENOCONV, STF_ENAN = range(8)
STATUS_NAMES = {0: "STF_OK", 1: "STF_EINVAL", 2: "STF_ENOMEM", 3: "STF_EDEVICE", 4: "STF_ESTATE",
                5: "STF_EPIVOT", 6: "STF_ENOCONV", 7: "STF_ENAN"}
STF_C128, STF_C64 = 0, 1
STF_X0_ZERO, STF_X0_USER, STF_X0_LEARNED = 0, 1, 2
ORDERS = {"additive": 0, "rows": 1, "rows_cols": 2, "diagonal": 3, "checker": 4}
KERNEL_CLASSES = ["assemble", "stencil", "front_asm", "front_lu", "sweep_fwd", "sweep_bwd",
                  "scatter", "arnoldi", "update", "nn"]


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("k0", C.c_double), ("pml", C.c_int32 * 4), ("pml_order", C.c_int32),
                ("pml_R", C.c_double), ("px", C.c_int32), ("py", C.c_int32),
                ("overlap", C.c_int32), ("local_pml", C.c_int32),
                ("local_pml_order", C.c_int32), ("local_pml_R", C.c_double),
                ("front_prec", C.c_int32), ("leaf_size", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32),
                ("x0_mode", C.c_int32), ("rounds", C.c_int32), ("debug_fault", C.c_int32),
                ("order", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("status", C.c_int32),
                ("history_len", C.c_int32), ("relres_true", C.c_double),
                ("relres_x0", C.c_double), ("history", C.POINTER(C.c_double)),
                ("history_cap", C.c_int32), ("used_learned", C.c_int32),
                ("t_factor_ms", C.c_double), ("t_solve_ms", C.c_double), ("t_nn_ms", C.c_double)]


class NNConfig(C.Structure):
    _fields_ = [("n", C.c_int32), ("width", C.c_int32), ("modes", C.c_int32),
                ("layers", C.c_int32), ("cin", C.c_int32), ("max_batch", C.c_int32)]


class TuneReport(C.Structure):
    _fields_ = [("levels", C.c_int32), ("changed", C.c_int32), ("ms_default", C.c_double),
                ("ms_tuned", C.c_double), ("fuse_depth", C.c_int32), ("ms_round_default", C.c_double),
                ("ms_round_tuned", C.c_double)]


class PlanInfo(C.Structure):
    _fields_ = [("ndof", C.c_int64), ("nsub", C.c_int32), ("nshapes", C.c_int32),
                ("local_dof", C.c_int64), ("nfronts", C.c_int64), ("max_front", C.c_int32),
                ("max_depth", C.c_int32), ("factor_entries", C.c_int64),
                ("front_entries", C.c_int64), ("lu_flops", C.c_double),
                ("device_bytes", C.c_int64)]


EXPORTS = {
    "stf_ctx_create": (C.c_int, [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "stf_ctx_destroy": (None, [C.c_void_p]),
    "stf_last_error": (C.c_char_p, [C.c_void_p]),
    "stf_ctx_set_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "stf_ctx_set_timing_mask": (C.c_int, [C.c_void_p, C.c_uint32]),
    "stf_ctx_kernel_stats": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double),
                                       C.POINTER(C.c_int64)]),
    "stf_plan_query": (C.c_int, [C.POINTER(Params), C.POINTER(PlanInfo)]),
    "stf_debug_local_axes": (C.c_int, [C.POINTER(Params), C.c_int32, C.POINTER(C.c_int32),
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "stf_problem_create": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_void_p, C.c_int,
                                     C.POINTER(C.c_void_p)]),
    "stf_assemble": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "stf_factor": (C.c_int, [C.c_void_p]),
    "stf_solve": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int,
                            C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
    "stf_factor_solve": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int,
                                   C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
    "stf_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "stf_precond_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "stf_precond_apply_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "stf_precond_apply_batch": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int]),
    "stf_stationary_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double,
                                       C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                       C.POINTER(C.c_int32)]),
    "stf_line_flux": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int32, C.c_int32, C.c_int32,
                                C.c_int32, C.POINTER(C.c_double)]),
    "stf_rcs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int32, C.c_void_p,
                          C.c_void_p, C.c_void_p]),
    "stf_sweep_apply": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int]),
    "stf_batch_solve": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_int, C.POINTER(SolveOpts), C.c_void_p]),
    "stf_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                               C.POINTER(TuneReport)]),
    "stf_debug_level_shapes": (C.c_int, [C.POINTER(Params), C.c_int32, C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "stf_tune_pick": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                C.POINTER(C.c_int32)]),
    "stf_tune_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "stf_tune_load": (C.c_int, [C.c_void_p, C.c_char_p]),
    "stf_tune_clear": (C.c_int, [C.c_void_p]),
    "stf_tune_count": (C.c_int32, [C.c_void_p]),
    "stf_tune_entry": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "stf_problem_info": (C.c_int, [C.c_void_p, C.POINTER(PlanInfo)]),
    "stf_problem_destroy": (None, [C.c_void_p]),
    "stf_nn_param_count": (C.c_int64, [C.POINTER(NNConfig)]),
    "stf_nn_create": (C.c_int, [C.c_void_p, C.POINTER(NNConfig), C.c_void_p,
                                C.POINTER(C.c_void_p)]),
    "stf_nn_destroy": (None, [C.c_void_p]),
    "stf_nn_get_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "stf_nn_set_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "stf_nn_forward": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "stf_nn_loss_grad": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.POINTER(C.c_double), C.c_void_p]),
    "stf_nn_train_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_double,
                                    C.c_int32, C.POINTER(C.c_double)]),
    "stf_ctx_set_nn": (C.c_int, [C.c_void_p, C.c_void_p]),
    "stf_nn_initial_guess": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "stf_nn_tile_data": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.POINTER(C.c_int32)]),
}

_lib = None


def load():
    """Load the HIP library; raises if it has not been built (there is no fallback).

    PyTorch (when installed) is imported first: its wheel carries its own HIP
    runtime, and loading ours first would put two HIP runtimes in one process.
    With torch loaded, the library binds to the runtime torch already holds.
    """
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libstfdfd.so is not built; run `python -m paper_2509_20801_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
