"""ctypes loader for libddm.so: declarations mirror include/ddm.h one to one.

The library is built in-tree (``python -m paper_2012_05695_amd.build``).  There
is no fallback: if the shared object is missing or fails to load, importing
the binding raises.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddm.so")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_uint32 = ctypes.c_uint32
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
P = ctypes.POINTER

DDM_OK = 0
DDM_ERR_INVALID_ARGUMENT = 1
DDM_ERR_UNSUPPORTED = 2
DDM_ERR_OUT_OF_MEMORY = 3
DDM_ERR_HIP = 4
DDM_ERR_STATE = 5
DDM_WARN_FP16_SATURATED = 100

DDM_KERNEL_ROW = 1
DDM_KERNEL_COL = 2
DDM_KERNEL_TIME = 4
DDM_KERNEL_RADIAL = 8
DDM_KERNEL_STEP1 = 16

DDM_NOALLOC_SCRATCH_BYTES = 256 << 20  # static device scratch of ddm_structure_function_noalloc

DDM_PIX_U8 = 1
DDM_PIX_U16 = 2
DDM_SPEC_F32 = 0
DDM_SPEC_F16_QSCALED = 1
DDM_PAD_POW2 = 0
DDM_PAD_MINIMAL = 1
DDM_METHOD_FOURIER = 0
DDM_METHOD_DIRECT = 1
DDM_METHOD_AUTO = 2

STATUS_NAMES = {
    0: "DDM_OK",
    1: "DDM_ERR_INVALID_ARGUMENT",
    2: "DDM_ERR_UNSUPPORTED",
    3: "DDM_ERR_OUT_OF_MEMORY",
    4: "DDM_ERR_HIP",
    5: "DDM_ERR_STATE",
    100: "DDM_WARN_FP16_SATURATED",
}


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("struct_size", c_uint32),
        ("width", c_int32),
        ("height", c_int32),
        ("n_frames", c_int32),
        ("max_lag", c_int32),
        ("pixel", c_int32),
        ("spectrum", c_int32),
        ("precondition", c_int32),
        ("padding", c_int32),
        ("method", c_int32),
        ("k2_max", c_int64),
        ("stream", c_void_p),
    ]


class FitDesc(ctypes.Structure):
    _fields_ = [
        ("struct_size", c_uint32),
        ("K", c_int32),
        ("max_iter", c_int32),
        ("fallback", c_int32),
        ("lambda0", ctypes.c_double),
        ("ftol", ctypes.c_double),
        ("xtol", ctypes.c_double),
        ("gtol", ctypes.c_double),
        ("stream", c_void_p),
    ]


DDM_FIT_CONVERGED = 1
DDM_FIT_MAXITER = 2
DDM_FIT_NONFINITE = 4
DDM_FIT_STALLED = 8
DDM_FIT_FALLBACK = 16
DDM_FIT_DEFAULT_START = 32

# (name, restype, argtypes) for every symbol of include/ddm.h
SIGNATURES = [
    ("ddm_plan_desc_init", None, [P(PlanDesc)]),
    ("ddm_plan_create", c_int32, [P(PlanDesc), P(c_void_p)]),
    ("ddm_plan_destroy", c_int32, [c_void_p]),
    ("ddm_plan_query", c_int32, [c_void_p, P(c_int64), P(c_int32), P(c_int32)]),
    ("ddm_plan_q_index", c_int32, [c_void_p, c_void_p, c_void_p]),
    ("ddm_plan_workspace_size", c_int32, [c_void_p, P(c_size_t), P(c_size_t)]),
    ("ddm_plan_set_workspace", c_int32, [c_void_p, c_void_p, c_size_t]),
    ("ddm_structure_function", c_int32, [c_void_p, c_void_p, c_void_p]),
    ("ddm_structure_function_noalloc", c_int32, [c_void_p, c_void_p, c_void_p]),
    ("ddm_structure_function_host", c_int32, [c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("ddm_image_spectra", c_int32, [c_void_p, c_void_p, c_void_p]),
    ("ddm_structure_from_spectra", c_int32, [c_void_p, c_void_p, c_void_p]),
    ("ddm_radial_average", c_int32,
     [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    ("ddm_plan_fp16_saturations", c_int32, [c_void_p, P(c_int64)]),
    ("ddm_plan_status", c_int32, [c_void_p]),
    ("ddm_plan_method", c_int32, [c_void_p, P(c_int32)]),
    ("ddm_plan_set_profiling", c_int32, [c_void_p, c_uint32]),
    ("ddm_plan_get_profile", c_int32, [c_void_p, c_uint32, P(ctypes.c_double), P(c_int64)]),
    ("ddm_sample_curves", c_int32,
     [c_void_p, c_int64, c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    ("ddm_fit_desc_init", None, [P(FitDesc)]),
    ("ddm_fit", c_int32, [P(FitDesc), c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("ddm_last_error", ctypes.c_char_p, []),
    ("ddm_abi_version", c_int32, []),
]


def load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(
            "libddm.so not found at %s; build it with `python -m paper_2012_05695_amd.build`" % path)
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib

DDM_MLP_IN = 64
DDM_MLP_HIDDEN = 256
DDM_MLP_OUT = 3
DDM_MLP_NPARAMS = 148995

SIGNATURES += [
    ("ddm_mlp_create", c_int32, [ctypes.c_uint64, c_int64, c_void_p, P(c_void_p)]),
    ("ddm_mlp_destroy", c_int32, [c_void_p]),
    ("ddm_mlp_set_params", c_int32, [c_void_p, c_void_p]),
    ("ddm_mlp_get_params", c_int32, [c_void_p, c_void_p]),
    ("ddm_mlp_get_state", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, P(c_int64)]),
    ("ddm_mlp_set_state", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64]),
    ("ddm_mlp_forward", c_int32, [c_void_p, c_void_p, c_int64, c_void_p]),
    ("ddm_mlp_gradient", c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    ("ddm_mlp_adam_step", c_int32, [c_void_p, ctypes.c_float]),
    ("ddm_mlp_train_step", c_int32, [c_void_p, c_void_p, c_void_p, c_int64, ctypes.c_float, c_void_p]),
]

SIGNATURES += [
    ("ddm_plan_autotune", c_int32, [c_void_p, P(c_int32), P(c_int32), P(ctypes.c_double)]),
    ("ddm_batch_create", c_int32, [P(PlanDesc), c_int32, c_int32, c_void_p, P(c_void_p)]),
    ("ddm_batch_destroy", c_int32, [c_void_p]),
    ("ddm_batch_query", c_int32, [c_void_p, c_int32, P(c_int64), P(c_int32), P(c_int32)]),
    ("ddm_batch_workspace_size", c_int32, [c_void_p, P(c_size_t)]),
    ("ddm_batch_set_workspace", c_int32, [c_void_p, c_void_p, c_size_t]),
    ("ddm_batch_autotune", c_int32, [c_void_p]),
    ("ddm_batch_structure_function", c_int32, [c_void_p, c_void_p, c_void_p]),
    ("ddm_batch_status", c_int32, [c_void_p, c_void_p]),
    ("ddm_batch_set_bins", c_int32, [c_void_p, c_int32, c_void_p, c_int32]),
    ("ddm_batch_structure_function_binned", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
]
