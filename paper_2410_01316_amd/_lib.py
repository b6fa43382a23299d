"""ctypes declarations of libfastsum.so (include/fastsum.h)."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libfastsum.so")

OK, EINVAL, ENOMEM, EDEVICE, ERANGE, EUNSUPPORTED, ESTATE = range(7)
KERNELS = {"gauss": 0, "laplace": 1, "energy": 2, "matern32": 3, "matern52": 4, "matern72": 5}
PROJ = {"fp32": 0, "bf16": 1}
FLAG_GRAD = 1
FLAG_MATERIALIZE = 2
FLAG_SORTED = 4
PHASES = ("project", "spread", "fftconv", "gather", "reduce", "backproject", "sort")


class Params(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32), ("P", ctypes.c_int32), ("n_ft", ctypes.c_int32),
        ("window_w", ctypes.c_int32), ("oversample", ctypes.c_int32),
        ("kernel", ctypes.c_int32), ("proj", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("scale", ctypes.c_double), ("T", ctypes.c_double),
        ("gmax_factor", ctypes.c_double), ("R", ctypes.c_double),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_double), ("beta", ctypes.c_double),
        ("n_grid", ctypes.c_int32), ("window_w", ctypes.c_int32),
        ("poly_degree", ctypes.c_int32), ("n_ft", ctypes.c_int32),
        ("n_max", ctypes.c_int64), ("m_max", ctypes.c_int64),
        ("proj", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("grid_lo", ctypes.c_int32), ("grid_nr", ctypes.c_int32),
        ("last_spread_chunks", ctypes.c_int32), ("last_gather_groups", ctypes.c_int32),
        ("fused", ctypes.c_int32),
    ]


class ProblemDesc(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("n_ft", ctypes.c_int32), ("scale", ctypes.c_double),
                ("R", ctypes.c_double), ("xi", ctypes.c_void_p), ("n_max", ctypes.c_int64),
                ("m_max", ctypes.c_int64)]


class ProblemIO(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("w", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("s", ctypes.c_void_p), ("N", ctypes.c_int64), ("M", ctypes.c_int64)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("spread_chunk", ctypes.c_int32),
                ("gather_group", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_st = ctypes.c_int

SIGNATURES = {
    "fastsum_plan_create": (_st, [ctypes.POINTER(Params), _vp, _i64, _i64, _vp, ctypes.POINTER(_vp)]),
    "fastsum_destroy": (None, [_vp]),
    "fastsum_exec": (_st, [_vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp]),
    "fastsum_grad": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "fastsum_grad_xyw": (_st, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "fastsum_check": (_st, [_vp]),
    "fastsum_get_info": (_st, [_vp, ctypes.POINTER(PlanInfo)]),
    "fastsum_host_tables": (_st, [ctypes.POINTER(Params), _vp, _vp, _vp]),
    "fastsum_debug_read": (_st, [_vp, ctypes.c_int32, _vp, _i64]),
    "fastsum_status_string": (ctypes.c_char_p, [_st]),
    "fastsum_profile": (_st, [_vp, ctypes.c_int32]),
    "fastsum_set_launch": (_st, [_vp, _i64, ctypes.c_int32]),
    "fastsum_batch_create": (_st, [ctypes.POINTER(Params), ctypes.POINTER(ProblemDesc), ctypes.c_int32,
                                   ctypes.POINTER(BatchTuning), _vp, ctypes.POINTER(_vp)]),
    "fastsum_batch_set_tuning": (_st, [_vp, ctypes.POINTER(BatchTuning)]),
    "fastsum_batch_exec": (_st, [_vp, ctypes.POINTER(ProblemIO), ctypes.c_int32, _vp]),
    "fastsum_batch_check": (_st, [_vp]),
    "fastsum_batch_destroy": (None, [_vp]),
    "fastsum_choose_nft": (_st, [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                 ctypes.c_double, ctypes.POINTER(ctypes.c_int32)]),
    "fastsum_profile_read": (_st, [_vp, _vp, _vp]),
    "fastsum_distance_qmc": (_st, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                   _vp, _vp]),
    "fastsum_bound": (_st, [_vp, _i64, _vp, _i64, ctypes.c_int32, _vp, ctypes.POINTER(ctypes.c_double)]),
    "fastsum_distance_qmc_noalloc": (_st, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_double, _vp, _vp]),
    "fastsum_rotate_directions": (_st, [ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp]),
    "fastsum_flow_update": (_st, [_i64, ctypes.c_int32, ctypes.c_float, ctypes.c_float, _vp, _vp,
                                  _vp, _vp, _vp, _vp]),
}

_lib = None


def load():
    """Load libfastsum.so once.  Raises ImportError when it is not built:
    there is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing; build it with `python -m paper_2410_01316_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class FastSumError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = load().fastsum_status_string(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")


def check(status, where):
    if status != OK:
        raise FastSumError(status, where)
