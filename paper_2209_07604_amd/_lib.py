"""ctypes declarations for libphi.so (the C ABI of include/phi.h).

Argument marshalling only.  Loading fails loudly when the library has not
been built: there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PHI_LIB") or os.path.join(HERE, "libphi.so")

PHI_OK = 0
STATUS = {
    0: "PHI_OK", -1: "PHI_ERR_ARG", -2: "PHI_ERR_SHAPE", -3: "PHI_ERR_RANGE",
    -4: "PHI_ERR_WORKSPACE", -5: "PHI_ERR_NONFINITE", -6: "PHI_ERR_HIP",
    -7: "PHI_ERR_UNSUPPORTED", -8: "PHI_ERR_STATE",
}
G_PREC = {"c64": 0, "f16": 1, "bf16": 2, "kb": 3}
HOST_C128, HOST_C64 = 0, 1
PER_CHANNEL, GRAPH, PERSISTENT, FUSED_GH, DR = 1, 2, 4, 8, 16

# every symbol include/phi.h declares
EXPORTS = [
    "phi_plan_create", "phi_plan_destroy", "phi_plan_workspace_size", "phi_plan_bind",
    "phi_plan_load_g", "phi_plan_set_theta", "phi_plan_get_info", "phi_plan_set_flags", "phi_plan_set_tuning", "phi_to_plan_order",
    "phi_from_plan_order", "phi_forward", "phi_adjoint", "l2ball_dual_step",
    "phi_plan_check", "phi_plan_set_timing", "phi_plan_get_timing", "phi_plan_autotune",
    "phi_status_string", "phi_dr_setup", "l2ball_dual_step_dr", "phi_dr_plan", "phi_dr_rows",
    "phi_psf", "phi_residual_image", "phi_power_iteration", "phi_plan_load_kb",
    "phi_pdfb_primal", "phi_eps_update", "phi_pdfb_run", "phi_plan_build_g", "phi_plan_read_g",
    "phi_power_iteration_static",
]


class PhiError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (where, STATUS.get(code, "?"), code))


class Desc(ctypes.Structure):
    _fields_ = [
        ("n_channels", ctypes.c_int32), ("ny", ctypes.c_int32), ("nx", ctypes.c_int32),
        ("h_n_blocks", ctypes.c_void_p), ("h_n_vis", ctypes.c_void_p),
        ("h_base", ctypes.c_void_p), ("h_stencil", ctypes.c_void_p),
        ("h_theta", ctypes.c_void_p), ("h_scale_y", ctypes.c_void_p),
        ("h_scale_x", ctypes.c_void_p), ("g_prec", ctypes.c_int32),
        ("flags", ctypes.c_int32), ("tile", ctypes.c_int32),
        ("persist_blocks", ctypes.c_int32),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("n_vis_total", ctypes.c_int64), ("n_taps", ctypes.c_int64),
        ("n_items", ctypes.c_int64), ("n_blocks_total", ctypes.c_int64),
        ("g_bytes", ctypes.c_int64), ("partial_bytes", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_int64), ("alg_bytes_dual_step", ctypes.c_double),
        ("alg_bytes_gather", ctypes.c_double), ("alg_bytes_scatter", ctypes.c_double),
        ("ky", ctypes.c_int32), ("kx", ctypes.c_int32), ("tile", ctypes.c_int32),
        ("n_stages", ctypes.c_int32), ("persist_blocks", ctypes.c_int32),
        ("fused", ctypes.c_int32), ("pitch_classes", ctypes.c_int32),
        ("dr_rows", ctypes.c_int64), ("dr_taps", ctypes.c_int64), ("dr_bytes", ctypes.c_int64),
        ("dr_max_window", ctypes.c_int32), ("reduced", ctypes.c_int32),
        ("fft_image_first", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class GBuild(ctypes.Structure):
    """phi_gbuild: Kaiser-Bessel width and the DDE table's shape."""
    _fields_ = [("J", ctypes.c_int32), ("n_ant", ctypes.c_int32), ("sa", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class EpsRule(ctypes.Structure):
    """phi_eps_rule: the adaptive l2-bound rule."""
    _fields_ = [
        ("lambda_lo", ctypes.c_double), ("lambda_hi", ctypes.c_double),
        ("lambda_mix", ctypes.c_double), ("var_tol", ctypes.c_double),
        ("min_gap", ctypes.c_int32), ("freeze", ctypes.c_int32),
    ]


_lib = None


def load():
    """The loaded libphi.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        # torch ships the HIP runtime under the same soname; load it first so
        # libphi and torch share one runtime (and one set of device pointers)
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libphi.so is not built (run __graft_entry__.build()); "
                           "there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    P, V, I32, I64, D = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "phi_plan_create": [ctypes.POINTER(Desc), ctypes.POINTER(P)],
        "phi_plan_destroy": [P],
        "phi_plan_workspace_size": [P, ctypes.POINTER(ctypes.c_size_t)],
        "phi_plan_bind": [P, V, ctypes.c_size_t, V],
        "phi_plan_load_g": [P, I64, V, I32, V],
        "phi_plan_set_theta": [P, V, V],
        "phi_plan_get_info": [P, ctypes.POINTER(Info)],
        "phi_plan_set_flags": [P, I32],
        "phi_plan_set_tuning": [P, I32, I32, V],
        "phi_to_plan_order": [P, V, V, V],
        "phi_from_plan_order": [P, V, V, V],
        "phi_forward": [P, V, V, V],
        "phi_adjoint": [P, V, V, V],
        "l2ball_dual_step": [P, V, V, V, V, V, V, V, V, V],
        "phi_plan_check": [P, V],
        "phi_plan_set_timing": [P, I32],
        "phi_plan_get_timing": [P, I32, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_char_p),
                                ctypes.POINTER(I32), ctypes.POINTER(I64)],
        "phi_plan_autotune": [P, V, I32],
        "phi_dr_setup": [P, V, V, V, V],
        "l2ball_dual_step_dr": [P, V, V, V, V, V, V, V, V, V],
        "phi_dr_plan": [P, ctypes.POINTER(P)],
        "phi_dr_rows": [P, V, V, V],
        "phi_plan_build_g": [P, I64, ctypes.POINTER(GBuild), V, V, V, V, V, V],
        "phi_plan_read_g": [P, I64, V, I32, V],
        "phi_power_iteration_static": [P, V, I32, V, V],
        "phi_pdfb_primal": [P, V, V, V, V, V, V],
        "phi_eps_update": [P, V, V, ctypes.POINTER(EpsRule), V, V, V],
        "phi_pdfb_run": [P, V, V, V, V, V, V, V, I32, ctypes.POINTER(EpsRule), V, V, V, V, V, V],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.phi_status_string.argtypes = [ctypes.c_int]
    lib.phi_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(code, where):
    if code != PHI_OK:
        raise PhiError(code, where)
