"""ctypes declarations of the C ABI in include/slmc.h (argument marshalling only)."""

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslmc.so")

SLMC_OK, SLMC_E_ARG, SLMC_E_SHAPE, SLMC_E_WORKSPACE, SLMC_E_DEVICE, SLMC_E_NONFINITE, \
    SLMC_E_UNSUPPORTED = range(7)
SLMC_FLAG_SERIAL = 1
SLMC_FLAG_STREAM_E = 2
SLMC_FP64, SLMC_FP32, SLMC_BF16X3, SLMC_BF16X6, SLMC_FP32_PLAIN, SLMC_INT8X5 = range(6)

EXPORTS = ("slmc_version", "slmc_last_error", "slmc_expk", "slmc_workspace_bytes", "slmc_logdet",
           "slmc_green", "slmc_eff_energy", "slmc_eff_sweep", "slmc_accept_workspace_bytes",
           "slmc_cumulative_accept", "slmc_log_weight", "slmc_profile", "slmc_profile_read",
           "slmc_profile_reset", "slmc_profile_name", "slmc_cache_clear", "slmc_green_noalloc",
           "slmc_eff_wolff", "slmc_eff_propose", "slmc_slices_workspace_bytes",
           "slmc_green_slices", "slmc_dqmc_workspace_bytes", "slmc_dqmc_sweep", "slmc_dqmc_block",
           "slmc_fit_workspace_bytes", "slmc_eff_fit", "slmc_step", "slmc_autotune",
           "slmc_tuning_lookup")
SLMC_NOALLOC_WORKSPACE_BYTES = 248 << 20


class Model(C.Structure):
    _fields_ = [("Lx", C.c_int32), ("Ly", C.c_int32), ("Ltau", C.c_int32), ("n_s", C.c_int32),
                ("t", C.c_double), ("mu", C.c_double), ("dtau", C.c_double),
                ("lam", C.c_double), ("omega0", C.c_double), ("c_kin", C.c_double)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("residual_steps", C.c_int32),
                ("acc_chunk", C.c_int32), ("flags", C.c_int32)]


class Batch(C.Structure):
    _fields_ = [("n_items", C.c_int32), ("model_idx", C.POINTER(C.c_int32)),
                ("x_off", C.POINTER(C.c_int64)), ("g_off", C.POINTER(C.c_int64))]


class Eff(C.Structure):
    _fields_ = [("Jk", C.c_double), ("J2", C.c_double), ("Jp", C.c_double), ("Jp6", C.c_double),
                ("a", C.c_double), ("Js", C.c_double * 3), ("Jt", C.c_double),
                ("delta", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("schedule", C.c_int32), ("seg_ahead", C.c_int32), ("gate", C.c_int32),
                ("seg_mode", C.c_int32), ("seg_cb", C.c_int32), ("ms_per_call", C.c_double)]


_lib = None


def lib():
    """Loads libslmc.so (built by ``__graft_entry__.build()``); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libslmc.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    vp, i32, u64, sz = C.c_void_p, C.c_int32, C.c_uint64, C.c_size_t
    P = C.POINTER
    L.slmc_version.restype = C.c_int
    L.slmc_last_error.restype = C.c_char_p
    L.slmc_expk.argtypes = [P(Model), P(C.c_double)]
    L.slmc_workspace_bytes.restype = sz
    L.slmc_workspace_bytes.argtypes = [P(Model), i32, P(Batch), P(Options)]
    L.slmc_logdet.argtypes = [P(Model), i32, P(Batch), P(Options), vp, vp, vp, vp, vp, sz, vp]
    L.slmc_green.argtypes = [P(Model), i32, P(Batch), P(Options), vp, vp, vp, vp, vp, vp, sz, vp]
    L.slmc_eff_energy.argtypes = [P(Model), P(Eff), i32, vp, vp, vp]
    L.slmc_eff_sweep.argtypes = [P(Model), P(Eff), i32, vp, i32, u64, u64, vp, vp]
    L.slmc_accept_workspace_bytes.restype = sz
    L.slmc_accept_workspace_bytes.argtypes = [P(Model), i32, P(Options)]
    L.slmc_cumulative_accept.argtypes = [P(Model), P(Eff), P(Options), i32, vp, vp, vp, vp, u64,
                                         u64, vp, vp, vp, vp, vp, sz, vp]
    L.slmc_profile.argtypes = [C.c_int]
    L.slmc_profile_read.argtypes = [i32, P(C.c_double), P(C.c_int64)]
    L.slmc_profile_reset.restype = None
    L.slmc_profile_name.restype = C.c_char_p
    L.slmc_profile_name.argtypes = [i32]
    L.slmc_log_weight.argtypes = [P(Model), P(Options), i32, vp, vp, vp, vp, sz, vp]
    L.slmc_cache_clear.restype = None
    L.slmc_slices_workspace_bytes.restype = sz
    L.slmc_slices_workspace_bytes.argtypes = [P(Model), i32, P(Options)]
    L.slmc_green_slices.argtypes = [P(Model), P(Options), i32, vp, i32, vp, vp, vp, vp, vp, sz, vp]
    L.slmc_dqmc_workspace_bytes.restype = sz
    L.slmc_dqmc_workspace_bytes.argtypes = [P(Model), i32, P(Options)]
    L.slmc_dqmc_sweep.argtypes = [P(Model), P(Options), i32, vp, C.c_double, i32, u64, u64, vp, vp, vp,
                                  vp, sz, vp]
    L.slmc_dqmc_block.argtypes = [P(Model), P(Options), i32, vp, vp, i32, u64, u64, vp, vp, vp, sz, vp]
    L.slmc_fit_workspace_bytes.restype = sz
    L.slmc_fit_workspace_bytes.argtypes = [i32]
    L.slmc_eff_fit.argtypes = [P(Model), C.c_double, i32, vp, vp, i32, vp, vp, vp, sz, vp]
    L.slmc_step.argtypes = [P(Model), P(Eff), P(Options), i32, vp, vp, vp, vp, i32, i32, u64, vp, vp, vp,
                            vp, vp, vp, vp, sz, vp]
    L.slmc_autotune.argtypes = [P(Model), P(Options), i32, vp, vp, sz, vp, P(Tuning), P(i32), P(i32)]
    L.slmc_tuning_lookup.argtypes = [P(Model), P(Options), i32, P(Tuning), P(i32)]
    L.slmc_eff_wolff.argtypes = [P(Model), P(Eff), i32, vp, i32, u64, u64, vp, vp]
    L.slmc_eff_propose.argtypes = [P(Model), P(Eff), i32, vp, i32, i32, u64, u64, vp, vp, vp]
    L.slmc_green_noalloc.argtypes = [P(Model), P(Options), i32, vp, vp, vp, vp, vp, vp]
    _lib = L
    return L


class SlmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("slmc error %d: %s" % (code, msg))
        self.code = code


def check(rc):
    if rc != SLMC_OK:
        raise SlmcError(rc, lib().slmc_last_error().decode())
    return rc
