"""ctypes mirror of include/dft.h.  Loading fails loudly when the HIP library is absent."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdftpicard.so")

MAX_SPECIES = 8
NALPHA = 10
NPASS = 10
PASS_NAMES = ["x_fwd", "y_fwd", "z_weights", "y_inv", "x_fmt", "y_fwd2", "z_back_es", "y_inv2",
              "x_el", "reduce"]

DFT_OK = 0
STATUS_NAMES = {0: "DFT_OK", 1: "DFT_E_INVALID_ARG", 2: "DFT_E_UNSUPPORTED_SIZE", 3: "DFT_E_WORKSPACE",
                4: "DFT_E_DEVICE", 5: "DFT_E_NONFINITE", 6: "DFT_E_PACKING", 7: "DFT_E_NOT_CONVERGED",
                8: "DFT_E_NOT_NEUTRAL"}
DFT_FP64 = 0
DFT_FP32_MIXED = 1
FLAG_ALLOW_NON_NEUTRAL = 1
FLAG_CUTOFF_LAMBDA = 2
FLAG_NO_AUTOTUNE = 4
HS_RSLT, HS_ROSENFELD, HS_WHITE_BEAR = 0, 1, 2
HS_FUNCTIONALS = {"rslt": HS_RSLT, "rosenfeld": HS_ROSENFELD, "whitebear": HS_WHITE_BEAR}
SCHEDULE_LEN = 12
ADJOINT_NOALLOC_MAX_BYTES = 64 << 20
RFD_MAX_NODES = 128
TUNE_PASSES = ["y", "z_plain", "z_weights", "z_back", "y_fwd2", "y_species"]

D8 = ctypes.c_double * MAX_SPECIES


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("h", ctypes.c_double * 3), ("nspecies", ctypes.c_int32),
                ("radius", D8), ("valence", D8), ("rho_bulk", D8), ("bjerrum_length", ctypes.c_double),
                ("electrostatics", ctypes.c_int32), ("precision", ctypes.c_int32), ("eta_cap", ctypes.c_double),
                ("flags", ctypes.c_int32), ("hs_functional", ctypes.c_int32)]


class BulkInfo(ctypes.Structure):
    _fields_ = [("mu_hs", D8), ("beta_p", ctypes.c_double), ("xi", ctypes.c_double * 4),
                ("gamma", ctypes.c_double), ("eta_msa", ctypes.c_double), ("omega", ctypes.c_double),
                ("lambda_", D8), ("mu_es", D8)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("rejected", ctypes.c_int64), ("g_evals", ctypes.c_int64),
                ("n3_evals", ctypes.c_int64), ("fp64_refresh", ctypes.c_int64), ("residual", ctypes.c_double),
                ("alpha", ctypes.c_double), ("max_n3", ctypes.c_double), ("step_cap", ctypes.c_double),
                ("compact_layout", ctypes.c_int32)]


class DftError(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
# (name, argtypes) in the order of include/dft.h
SIGNATURES = [
    ("dft_last_error", []),
    ("dft_bulk", [ctypes.POINTER(Params), ctypes.POINTER(BulkInfo)]),
    ("dft_workspace_size", [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]),
    ("dft_setup", [ctypes.POINTER(Params), _vp, _vp, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    ("dft_set_stream", [_vp, _vp]),
    ("dft_residual", [_vp, _vp, _vp, _dp]),
    ("dft_operators", [_vp, _vp, _vp, _vp, _vp, _vp]),
    ("dft_set_reference", [_vp, _vp]),
    ("dft_picard_step", [_vp, _vp, _dp, _dp]),
    ("dft_solve", [_vp, _vp, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _dp]),
    ("dft_run", [_vp, _vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _dp]),
    ("dft_profile", [_vp, _vp, ctypes.c_int32, _dp]),
    ("dft_adjoint_workspace_size", [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]),
    ("dft_adjoint", [_vp, _vp, _vp, _vp, ctypes.c_size_t, ctypes.c_double, ctypes.c_int32, _vp, _dp, _dp,
                     ctypes.POINTER(ctypes.c_int32), _dp]),
    ("dft_adjoint_noalloc", [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int32, _vp, _dp, _dp,
                             ctypes.POINTER(ctypes.c_int32), _dp]),
    ("dft_batch_workspace_size", [ctypes.POINTER(Params), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    ("dft_setup_batch", [ctypes.POINTER(Params), ctypes.c_int32, _vp, _vp, _vp, ctypes.c_size_t, _vp,
                         ctypes.POINTER(_vp)]),
    ("dft_batch_member", [_vp, ctypes.c_int32, ctypes.POINTER(_vp)]),
    ("dft_solve_batch", [_vp, _vp, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _dp,
                         ctypes.POINTER(ctypes.c_int32)]),
    ("dft_batch_destroy", [_vp]),
    ("dft_get_stats", [_vp, ctypes.POINTER(Stats)]),
    ("dft_newton", [_vp, _vp, _vp, ctypes.c_size_t, ctypes.c_double, ctypes.c_int32,
                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _dp]),
    ("dft_rfd_reference", [_vp, _vp, _vp, ctypes.c_int32, _vp]),
    ("dft_get_schedule", [_vp, ctypes.POINTER(ctypes.c_int32)]),
    ("dft_set_schedule", [_vp, ctypes.POINTER(ctypes.c_int32)]),
    ("dft_destroy", [_vp]),
]

_lib = None


def load():
    """Load libdftpicard.so (built by paper_0910_1531_amd.build); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_0910_1531_amd.build`; "
                          "there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "dft_last_error" else ctypes.c_int
    _lib = lib
    return lib


def check(status, where):
    if status != DFT_OK:
        raise DftError(status, where, load().dft_last_error().decode())
    return status
