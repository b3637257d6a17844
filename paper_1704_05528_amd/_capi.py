"""ctypes declarations of the C-ABI in include/svt.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))

SVT_OK = 0
SVT_E_INVALID_ARG, SVT_E_OOM, SVT_E_HIP, SVT_E_NUMERIC, SVT_E_STATE, SVT_E_LIMIT = -1, -2, -3, -4, -5, -6
SVT_GRAD_FROZEN_BASIS, SVT_GRAD_DEVICE_POINTERS = 1, 2
SVT_DTYPE_F64, SVT_DTYPE_F32 = 0, 1
SVT_FP64, SVT_MIXED, SVT_BF16 = 0, 1, 2
SVT_MODE_R4SVD, SVT_MODE_R3SVD, SVT_MODE_RSVD = 0, 1, 2
SVT_F_CONVERGED, SVT_F_MAXIT, SVT_F_RMAX_HIT, SVT_F_EXHAUSTED, SVT_F_ANNEALED, SVT_F_EIG_INEXACT = 1, 2, 4, 8, 16, 32
SVT_F_DIVERGING = 64

_STATUS = {0: "SVT_OK", -1: "SVT_E_INVALID_ARG", -2: "SVT_E_OOM", -3: "SVT_E_HIP", -4: "SVT_E_NUMERIC",
           -5: "SVT_E_STATE", -6: "SVT_E_LIMIT"}

# Names of every symbol include/svt.h declares (checked by the CPU tests).
EXPORTS = ["svt_default_params", "svt_init", "r4svd_step", "svt_iterate", "svt_history", "svt_factors", "svt_sample",
           "svt_mae", "svt_mae_device", "svt_get_state", "svt_set_state", "svt_checkpoint", "svt_restore",
           "svt_set_replay", "svt_grad", "svt_profile",
           "svt_profile_phases", "svt_profile_read", "svt_time_phase", "svt_last_error", "svt_destroy"]
PHASES = ["spmm_t", "grow", "gram", "eig", "factors", "sddmm", "reduce", "densify"]


class SVTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("tau", C.c_double), ("delta", C.c_double), ("tol", C.c_double), ("beta", C.c_double),
                ("eta", C.c_double), ("eps_thr0", C.c_double), ("maxit", C.c_int32), ("t0", C.c_int32),
                ("dt", C.c_int32), ("npow", C.c_int32), ("r_max", C.c_int32), ("k0", C.c_int32),
                ("seed", C.c_uint64), ("precision", C.c_int32), ("kmax", C.c_int32), ("mode", C.c_int32),
                ("recycle_extra", C.c_int32), ("rank", C.c_int32), ("oversample", C.c_int32),
                ("mae_tol", C.c_double), ("wait_timeout_s", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("iter", C.c_int32), ("r", C.c_int32), ("k", C.c_int32), ("blocks", C.c_int32),
                ("annealed", C.c_int32), ("stopped", C.c_int32), ("flags", C.c_int32), ("eig_iters", C.c_int32),
                ("eps", C.c_double), ("eps_thr", C.c_double), ("rel_res", C.c_double), ("normY", C.c_double),
                ("normB", C.c_double), ("sigma1", C.c_double), ("sigmak", C.c_double),
                ("grow_margin", C.c_double), ("anneal_margin", C.c_double), ("mae", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = C.POINTER
_i32p, _f64p, _vp = _P(C.c_int32), _P(C.c_double), C.c_void_p
_lib = None


def lib_path():
    return os.path.join(HERE, "libsvt.so")


def load():
    """Load libsvt.so from this package folder; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise SVTError(SVT_E_STATE, f"{path} is missing: build it with `python -m paper_1704_05528_amd.build`")
    # torch bundles its own HIP runtime (same soname as /opt/rocm's).  Importing torch first makes
    # libsvt bind to that already-loaded runtime, so the process holds a single HIP runtime and
    # torch tensors, streams and this library see the same devices.
    import torch  # noqa: F401
    L = C.CDLL(path)
    L.svt_default_params.argtypes = [_P(Params)]
    L.svt_default_params.restype = None
    # pointers that may be host or device memory (by a flag of the call) are declared void*
    L.svt_init.argtypes = [_P(_vp), C.c_int64, C.c_int64, C.c_int64, _vp, _vp, _vp, C.c_int32, C.c_int32,
                           _P(Params), _vp]
    L.r4svd_step.argtypes = [_vp, _P(StepStats)]
    L.svt_iterate.argtypes = [_vp, C.c_int32, _P(StepStats)]
    L.svt_history.argtypes = [_vp, C.c_int64, C.c_int64, _P(StepStats), _P(C.c_int64)]
    L.svt_factors.argtypes = [_vp, C.c_int32, _i32p, _vp, _vp, _vp, C.c_int32]
    L.svt_sample.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, C.c_int32]
    L.svt_mae.argtypes = [_vp, C.c_int64, _i32p, _i32p, _f64p, _f64p]
    L.svt_get_state.argtypes = [_vp, _f64p, _f64p, C.c_int32, _i32p, _f64p, _f64p, _i32p]
    L.svt_set_state.argtypes = [_vp, _f64p, _f64p, C.c_int32, C.c_double, C.c_double, C.c_int32]
    L.svt_set_replay.argtypes = [_vp, _i32p, _i32p, C.c_int32]
    L.svt_grad.argtypes = [_vp, C.c_int32, C.c_int32, C.c_int64, _vp, _vp, _vp, C.c_int32, _f64p, _f64p, _vp]
    L.svt_profile.argtypes = [_vp, C.c_int32]
    L.svt_profile_phases.argtypes = [_vp, C.c_uint32]
    L.svt_profile_read.argtypes = [_vp, _f64p, _f64p, _f64p, _P(C.c_int64)]
    L.svt_time_phase.argtypes = [_vp, C.c_int32, C.c_int32, _f64p, _f64p, _f64p]
    L.svt_checkpoint.argtypes = [_vp, C.c_void_p, C.c_int64, _P(C.c_int64)]
    L.svt_restore.argtypes = [_vp, C.c_void_p, C.c_int64]
    # device pointers (integers, e.g. torch.Tensor.data_ptr())
    L.svt_mae_device.argtypes = [_vp, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.svt_last_error.argtypes = [_vp]
    L.svt_last_error.restype = C.c_char_p
    L.svt_destroy.argtypes = [_vp]
    L.svt_destroy.restype = None
    for name in ["svt_init", "r4svd_step", "svt_iterate", "svt_history", "svt_factors", "svt_sample", "svt_mae",
                 "svt_mae_device", "svt_checkpoint", "svt_restore", "svt_get_state",
                 "svt_set_state", "svt_set_replay", "svt_grad", "svt_profile", "svt_profile_phases",
                 "svt_profile_read", "svt_time_phase"]:
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def require_gpu():
    """Raise unless libsvt.so is built and a ROCm GPU is visible."""
    load()
    import torch
    if not torch.cuda.is_available() or torch.version.hip is None:
        raise SVTError(SVT_E_STATE, "no ROCm GPU visible: the SVT library has no CPU path")


def default_params(**kw):
    p = Params()
    load().svt_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def check(status, handle=None):
    if status != SVT_OK:
        msg = load().svt_last_error(handle).decode(errors="replace")
        raise SVTError(status, msg)
