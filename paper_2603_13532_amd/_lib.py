"""ctypes view of the C ABI declared in include/tsk.h.

Argument marshalling only: structures, prototypes and the loader.  Loading
fails loudly (RuntimeError) when libtsk.so has not been built; there is no
fallback implementation anywhere in the package.
"""
import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_uint64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtsk.so")

# tsk_status
TSK_OK = 0
STATUS_NAMES = {
    0: "TSK_OK", 1: "TSK_ERR_INVALID_ARG", 2: "TSK_ERR_UNSUPPORTED", 3: "TSK_ERR_OUT_OF_MEMORY",
    4: "TSK_ERR_WORKSPACE_TOO_SMALL", 5: "TSK_ERR_DEVICE", 6: "TSK_ERR_RANK_DEFICIENT",
}
# tsk_dtype
TSK_F64, TSK_F32 = 0, 1
# tsk_sketch_kind
KINDS = {"krp": 0, "kron": 1}
# tsk_precision
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x1": 2, "bf16x3": 3, "bf16x6": 4}
QR_POLICIES = {"auto": 0, "householder": 1, "cholqr2": 2}


class TuckerSum(ctypes.Structure):
    _fields_ = [
        ("order", c_int32),
        ("num_terms", c_int32),
        ("dims", POINTER(c_int64)),
        ("ranks", POINTER(c_int32)),
        ("cores", POINTER(c_void_p)),
        ("factors", POINTER(c_void_p)),
        ("coeffs", POINTER(c_double)),
        ("dtype", c_int),
    ]


class SketchSpec(ctypes.Structure):
    _fields_ = [
        ("kind", c_int),
        ("sizes", POINTER(c_int32)),
        ("seed", c_uint64),
        ("omega", POINTER(c_void_p)),
        ("sketch_prec", c_int),
        ("project_prec", c_int),
        ("qr_policy", c_int32),
    ]


class Truncation(ctypes.Structure):
    _fields_ = [
        ("order", c_int32),
        ("dims", POINTER(c_int64)),
        ("widths", POINTER(c_int64)),
        ("Q", POINTER(c_void_p)),
        ("H", c_void_p),
        ("eps", c_double),
        ("U_out", POINTER(c_void_p)),
        ("G_out", c_void_p),
        ("ranks_out", POINTER(c_int32)),
    ]


# name -> (restype, argtypes); every function declared in include/tsk.h
PROTOTYPES = {
    "tsk_create": (c_int, [POINTER(c_void_p), c_int]),
    "tsk_destroy": (c_int, [c_void_p]),
    "tsk_status_string": (c_char_p, [c_int]),
    "tsk_last_error_detail": (c_char_p, [c_void_p]),
    "tsk_krp_width": (c_int, [c_int32, POINTER(c_int32), POINTER(c_int32)]),
    "tsk_kron_sizes": (c_int, [c_int32, POINTER(c_int32), POINTER(c_int32)]),
    "tsk_sketch_widths": (c_int, [POINTER(TuckerSum), POINTER(SketchSpec), POINTER(c_int64),
                                  POINTER(c_int64)]),
    "tsk_sketch_omega": (c_int, [c_void_p, c_uint64, c_int32, c_int64, c_int64, c_void_p, c_int,
                                 c_void_p]),
    "tucker_sum_workspace_size": (c_int, [c_void_p, POINTER(TuckerSum), POINTER(SketchSpec),
                                          POINTER(c_size_t)]),
    "tucker_sum_sketch": (c_int, [c_void_p, POINTER(TuckerSum), POINTER(SketchSpec),
                                  POINTER(c_void_p), c_void_p, c_size_t, c_void_p]),
    "tucker_sum_recompress": (c_int, [c_void_p, POINTER(TuckerSum), POINTER(SketchSpec),
                                      POINTER(c_void_p), c_void_p, c_int, POINTER(c_void_p),
                                      c_void_p, c_size_t, c_void_p]),
    "tucker_sum_project_workspace_size": (c_int, [c_void_p, POINTER(TuckerSum), POINTER(c_int64),
                                                  c_int, c_int, POINTER(c_size_t)]),
    "tucker_sum_project": (c_int, [c_void_p, POINTER(TuckerSum), POINTER(c_void_p),
                                   POINTER(c_int64), c_int, c_int, c_void_p, c_int, c_void_p,
                                   c_size_t, c_void_p]),
    "tucker_sum_subranks_workspace_size": (c_int, [c_void_p, POINTER(TuckerSum),
                                                   POINTER(c_size_t)]),
    "tucker_sum_subranks": (c_int, [c_void_p, POINTER(TuckerSum), c_double, POINTER(c_int32),
                                    POINTER(c_int32), c_void_p, c_size_t, c_void_p]),
    "tucker_sum_subranks_batched_workspace_size": (c_int, [c_void_p, c_int32, POINTER(TuckerSum),
                                                           POINTER(c_size_t)]),
    "tucker_sum_subranks_batched": (c_int, [c_void_p, c_int32, POINTER(TuckerSum), c_double,
                                            POINTER(c_int32), POINTER(c_int32), c_void_p,
                                            c_size_t, c_void_p]),
    "tucker_truncate_batched_workspace_size": (c_int, [c_void_p, c_int32, POINTER(Truncation),
                                                       POINTER(c_size_t)]),
    "tucker_truncate_batched": (c_int, [c_void_p, c_int32, POINTER(Truncation), c_void_p,
                                        c_size_t, c_void_p]),
    "tucker_truncate_workspace_size": (c_int, [c_void_p, c_int32, POINTER(c_int64),
                                               POINTER(c_int64), c_double, POINTER(c_size_t)]),
    "tucker_truncate": (c_int, [c_void_p, c_int32, POINTER(c_int64), POINTER(c_int64),
                                POINTER(c_void_p), c_void_p, c_double, POINTER(c_void_p),
                                c_void_p, POINTER(c_int32), c_void_p, c_size_t, c_void_p]),
    "tucker_sum_round_deterministic_workspace_size": (c_int, [c_void_p, POINTER(TuckerSum),
                                                              c_double, POINTER(c_size_t)]),
    "tucker_sum_round_deterministic": (c_int, [c_void_p, POINTER(TuckerSum), c_double,
                                               POINTER(c_void_p), c_void_p, POINTER(c_int32),
                                               c_void_p, c_size_t, c_void_p]),
    "tucker_sum_recompress_noalloc": (c_int, [c_void_p, POINTER(TuckerSum), POINTER(SketchSpec),
                                              POINTER(c_void_p), c_void_p, c_int,
                                              POINTER(c_void_p), c_void_p]),
    "tsk_qr_fallback_count": (c_int, [c_void_p, c_void_p, POINTER(c_int64)]),
    "tucker_sum_batched_workspace_size": (c_int, [c_void_p, c_int32, POINTER(TuckerSum),
                                                  POINTER(SketchSpec), POINTER(c_size_t)]),
    "tucker_sum_recompress_batched": (c_int, [c_void_p, c_int32, POINTER(TuckerSum),
                                              POINTER(SketchSpec), POINTER(POINTER(c_void_p)),
                                              POINTER(c_void_p), c_int, c_void_p, c_size_t,
                                              c_void_p]),
    "tucker_sum_backward_workspace_size": (c_int, [c_void_p, POINTER(TuckerSum),
                                                   POINTER(SketchSpec), POINTER(c_size_t)]),
    "tucker_sum_recompress_backward": (c_int, [c_void_p, POINTER(TuckerSum), POINTER(SketchSpec),
                                               POINTER(c_void_p), POINTER(c_void_p), c_void_p,
                                               POINTER(c_void_p), c_int, POINTER(c_void_p),
                                               POINTER(c_void_p), c_void_p, c_size_t, c_void_p]),
    "tsk_autotune": (c_int, [c_void_p, c_int32, POINTER(TuckerSum), POINTER(SketchSpec),
                             POINTER(POINTER(c_void_p)), POINTER(c_void_p), c_int, c_int32,
                             c_void_p]),
    "tsk_autotune_save": (c_int, [c_void_p, c_char_p]),
    "tsk_autotune_load": (c_int, [c_void_p, c_char_p]),
    "tsk_autotune_clear": (c_int, [c_void_p]),
    "tsk_profile_enable": (c_int, [c_void_p, c_int32]),
    "tsk_profile_report": (c_int, [c_void_p, c_char_p, c_size_t, POINTER(c_size_t)]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libtsk.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2603_13532_amd.build` (there is no fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class TskError(RuntimeError):
    def __init__(self, status, detail=""):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{self.name}: {detail}" if detail else self.name)


def check(status, handle=None):
    if status != TSK_OK:
        detail = ""
        if handle is not None:
            raw = load().tsk_last_error_detail(handle)
            detail = raw.decode() if raw else ""
        raise TskError(status, detail)
