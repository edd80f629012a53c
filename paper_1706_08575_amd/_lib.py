"""ctypes binding of libftcg (include/ftcg.h): the C entry points under the
same names, argument marshalling only. Every step of the path runs in the
library's HIP kernels; nothing here computes.

The library is loaded from this package directory. If it is missing the
import fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libftcg.so")

FTCG_OK, FTCG_EINVAL, FTCG_ENOMEM, FTCG_EHIP, FTCG_ESTATE, FTCG_EUNSUPPORTED = range(6)
FTCG_F64, FTCG_F32 = 0, 1
FTCG_W_PLAIN, FTCG_W_LEARNED, FTCG_W_USER, FTCG_W_NONE, FTCG_W_BAND, FTCG_W_DENSITY = range(6)
FTCG_ACCUM_FIXED, FTCG_ACCUM_F64 = 0, 1

STEP_NAMES = ("bin", "weights", "spread", "fft1", "fft2_deapod", "weight_bin", "learned", "audit",
              "weight_finish", "band_gram", "band_solve", "band_apply", "forward_fft", "forward_interp", "density", "frame_approx")
TIMING_STEPS = 16


class FtcgError(RuntimeError):
    def __init__(self, status: int, call: str):
        self.status = status
        super().__init__(f"{call}: {status_string(status)}")


_lib = None

# (name, restype, argtypes)
_SIGS = [
    ("ftcg_status_string", C.c_char_p, [C.c_int]),
    ("ftcg_plan_create", C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int64), C.c_int, C.c_double,
                                   C.c_int, C.c_int, C.c_double, C.c_void_p]),
    ("ftcg_plan_destroy", C.c_int, [C.c_void_p]),
    ("ftcg_set_points", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p]),
    ("ftcg_set_weights", C.c_int, [C.c_void_p, C.c_void_p]),
    ("ftcg_get_weights", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int)]),
    ("ftcg_execute", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ftcg_spread_only", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ftcg_grid_to_image", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ftcg_forward", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ftcg_frame_approx", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ftcg_plan_set_band", C.c_int, [C.c_void_p, C.c_int]),
    ("ftcg_plan_set_density_iterations", C.c_int, [C.c_void_p, C.c_int]),
    ("ftcg_get_band", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int)]),
    ("ftcg_grid_to_image_noalloc", C.c_int, [C.c_int, C.c_int64, C.c_int, C.c_double, C.c_int, C.c_void_p,
                                             C.c_void_p, C.c_void_p]),
    ("ftcg_plan_info", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int)]),
    ("ftcg_plan_set_tuning", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int]),
    ("ftcg_plan_set_spread_layout", C.c_int, [C.c_void_p, C.c_int]),
    ("ftcg_plan_set_weight_tuning", C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    ("ftcg_plan_enable_timing", C.c_int, [C.c_void_p, C.c_int]),
    ("ftcg_plan_timing", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    ("ftcg_mlp_create", C.c_int, [C.POINTER(C.c_void_p), C.c_void_p]),
    ("ftcg_mlp_destroy", C.c_int, [C.c_void_p]),
    ("ftcg_mlp_set_params", C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    ("ftcg_mlp_get_params", C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    ("ftcg_mlp_save", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)]),
    ("ftcg_mlp_load", C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    ("ftcg_mlp_features", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    ("ftcg_mlp_forward", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    ("ftcg_mlp_loss_grad", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                     C.POINTER(C.c_double)]),
    ("ftcg_mlp_train_batch", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int, C.c_float,
                                       C.POINTER(C.c_double)]),
    ("ftcg_mlp_train_raster", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_double, C.c_int64, C.c_float,
                                        C.c_int, C.POINTER(C.c_double)]),
    ("ftcg_plan_set_mlp", C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_int64]),
    ("ftcg_plan_learned_report", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    ("ftcg_batch_create", C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int64), C.c_int, C.c_double,
                                    C.c_int, C.c_double, C.c_void_p]),
    ("ftcg_batch_destroy", C.c_int, [C.c_void_p]),
    ("ftcg_batch_set_tuning", C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int, C.c_int]),
    ("ftcg_batch_set_mlp", C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_int64]),
    ("ftcg_batch_set_points", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_void_p]),
    ("ftcg_batch_set_weights", C.c_int, [C.c_void_p, C.c_void_p]),
    ("ftcg_batch_get_weights", C.c_int, [C.c_void_p, C.c_void_p]),
    ("ftcg_batch_execute", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ftcg_batch_info", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int64)]),
    ("ftcg_batch_enable_timing", C.c_int, [C.c_void_p, C.c_int]),
]

EXPORTED = [s[0] for s in _SIGS]
MLP_NPARAM = 6337


def lib() -> C.CDLL:
    """Load libftcg.so (once). Raises ImportError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().ftcg_status_string(int(s)).decode()


def check(status: int, call: str) -> None:
    if status != FTCG_OK:
        raise FtcgError(status, call)


def call(name: str, *args) -> int:
    """Call entry point ``name`` and return its raw status."""
    return getattr(lib(), name)(*args)
