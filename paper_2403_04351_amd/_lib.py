"""ctypes view of include/ltd.h (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# LTD_LIBRARY: another build of the same library (e.g. the host-sanitized one)
LIB_PATH = os.environ.get("LTD_LIBRARY") or os.path.join(HERE, "libltd.so")

LTD_OK = 0
LTD_EINVAL = -1
LTD_ESHAPE = -2
LTD_EALIGN = -3
LTD_ESTATE = -4
LTD_EWORKSPACE = -5
LTD_EUNSUPPORTED = -6
LTD_ESTEP = -7
LTD_EHIP = 1
LTD_ENOTSPD = 2
LTD_ENONFINITE = 3
LTD_ESPECTRUM = 4
LTD_ECAPTURE = 5

LTD_FP64 = 0
LTD_FP32_RESID = 1
LTD_BF16X3_RESID = 2
LTD_PULSE_GAUSS_SIN = 0
LTD_PULSE_SIN2 = 1
LTD_PULSE_KICK = 2
LTD_ROUTE_FFT = 0
LTD_ROUTE_MM = 1
LTD_ROUTE_FFT_PLANES = 2
LTD_STEP_REBUILD = 0
LTD_STEP_AFFINE = 1

EXPORTED = [
    "ltd_create", "ltd_bind_workspace", "ltd_destroy", "ltd_status_string", "ltd_sync_status",
    "ltd_apply_HS", "ltd_apply_HS_static", "ltd_project_subspace", "ltd_ritz_basis", "ltd_subspace_info",
    "ltd_propagate_step", "ltd_propagate", "ltd_propagate_prepare", "ltd_propagate_step_adjoint", "ltd_knot_samples",
    "ltd_knot_gradient", "ltd_chebyshev_coefficients", "ltd_profile_steps", "ltd_profile_apply",
    "ltd_rebuild_grid", "ltd_autotune", "ltd_set_tuning", "ltd_state_drift",
    "ltd_pulse_samples", "ltd_polarizability", "ltd_pulse_loss", "ltd_propagate_full", "ltd_full_spectrum",
]
LTD_PROFILE_STAGES = 8


class SystemDesc(C.Structure):
    _fields_ = [
        ("n_k", C.c_int),
        ("n_g", C.POINTER(C.c_int)),
        ("g_int", C.POINTER(C.c_int32)),
        ("gk_cart", C.POINTER(C.c_double)),
        ("grid", C.c_int * 3),
        ("theta_r", C.c_void_p),
        ("v_r", C.c_void_p),
        ("n_atoms", C.c_int),
        ("n_mt", C.POINTER(C.c_int)),
        ("n_lo", C.POINTER(C.c_int)),
        ("amat", C.c_void_p),
        ("h", C.c_void_p),
        ("o", C.c_void_p),
        ("pz", C.c_void_p),
        ("omega", C.c_double),
        ("c_light", C.c_double),
        ("occ", C.c_double),
        ("k_weight", C.POINTER(C.c_double)),
        ("n_aux", C.c_int),
        ("n_states", C.c_int),
        ("max_cols", C.c_int),
        ("interstitial_route", C.c_int),
    ]


class StepArgs(C.Structure):
    _fields_ = [
        ("mode", C.c_int),
        ("dt", C.c_double),
        ("a_t", C.c_void_p),
        ("a_mid", C.c_void_p),
        ("step", C.c_void_p),
        ("v_r_t", C.c_void_p),
        ("h_t", C.c_void_p),
        ("theta", C.c_void_p),
        ("c_out", C.c_void_p),
        ("j_out", C.c_void_p),
        ("e_out", C.c_void_p),
        ("dmu_out", C.c_void_p),
        ("v_stride", C.c_longlong),
        ("h_stride", C.c_longlong),
        ("taylor_order", C.c_int),
        ("nexc_out", C.c_void_p),
        ("theta_hist", C.c_void_p),
        ("hist_len", C.c_int),
    ]


class FullArgs(C.Structure):
    _fields_ = [
        ("dt", C.c_double),
        ("order", C.c_int),
        ("c0", C.c_double),
        ("a_mid", C.POINTER(C.c_double)),
        ("cg_max_iter", C.c_int),
        ("cg_tol", C.c_double),
        ("cg_resid", C.POINTER(C.c_double)),
        ("cg_iters", C.POINTER(C.c_int)),
    ]


class AdjointArgs(C.Structure):
    _fields_ = [
        ("fwd", C.POINTER(StepArgs)),
        ("n", C.c_int),
        ("terminal", C.c_int),
        ("n_steps", C.c_int),
        ("mu_next", C.c_void_p),
        ("mu_out", C.c_void_p),
        ("dl_da_mid", C.c_void_p),
        ("dl_da_t", C.c_void_p),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Loads libltd.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2403_04351_amd/build.py "
                           "(the HIP library is the only implementation)")
    lib = C.CDLL(path)
    vp, ip, dp = C.c_void_p, C.c_int, C.POINTER(C.c_double)
    lib.ltd_create.argtypes = [C.POINTER(SystemDesc), ip, C.POINTER(C.c_size_t), C.POINTER(vp)]
    lib.ltd_bind_workspace.argtypes = [vp, vp, C.c_size_t, vp]
    lib.ltd_destroy.argtypes = [vp]
    lib.ltd_status_string.argtypes = [ip]
    lib.ltd_status_string.restype = C.c_char_p
    lib.ltd_sync_status.argtypes = [vp, vp]
    lib.ltd_apply_HS.argtypes = [vp, ip, dp, vp, ip, ip, vp, ip, vp, ip, vp]
    lib.ltd_apply_HS_static.argtypes = [vp, ip, dp, vp, ip, ip, vp, ip, vp, ip, vp]
    lib.ltd_project_subspace.argtypes = [vp, ip, vp, ip, ip, vp, vp, vp, ip, ip, vp, vp]
    lib.ltd_ritz_basis.argtypes = [vp, ip, vp, ip, vp, vp]
    lib.ltd_subspace_info.argtypes = [vp, ip, dp, dp, dp]
    lib.ltd_rebuild_grid.argtypes = [vp, C.POINTER(ip)]
    lib.ltd_autotune.argtypes = [vp, C.POINTER(ip), dp, vp]
    lib.ltd_set_tuning.argtypes = [vp, C.POINTER(ip)]
    lib.ltd_state_drift.argtypes = [vp, vp, ip, dp, vp]
    lib.ltd_propagate_step.argtypes = [vp, C.POINTER(StepArgs), vp]
    lib.ltd_propagate.argtypes = [vp, C.POINTER(StepArgs), ip, vp]
    lib.ltd_propagate_prepare.argtypes = [vp, C.POINTER(StepArgs), ip, vp]
    lib.ltd_propagate_step_adjoint.argtypes = [vp, C.POINTER(AdjointArgs), vp]
    lib.ltd_knot_samples.argtypes = [vp, ip, C.c_double, C.c_double, ip, vp, vp, vp]
    lib.ltd_knot_gradient.argtypes = [vp, vp, ip, C.c_double, ip, C.c_double, vp, vp]
    lib.ltd_pulse_loss.argtypes = [vp, vp, ip, vp, vp]
    lib.ltd_propagate_full.argtypes = [vp, ip, vp, ip, ip, C.POINTER(FullArgs), ip, vp]
    lib.ltd_full_spectrum.argtypes = [vp, ip, vp, ip, ip, C.c_double, dp, vp]
    lib.ltd_pulse_samples.argtypes = [ip, dp, C.c_double, ip, vp, vp, vp]
    lib.ltd_polarizability.argtypes = [vp, vp, ip, C.c_double, C.c_double, C.c_double, vp, ip, C.c_double, vp, vp]
    lib.ltd_chebyshev_coefficients.argtypes = [C.c_double, ip, dp, C.POINTER(ip)]
    lib.ltd_profile_steps.argtypes = [vp, C.POINTER(StepArgs), ip, dp, vp]
    lib.ltd_profile_apply.argtypes = [vp, ip, vp, ip, ip, vp, vp, ip, dp, vp]
    for name in EXPORTED:
        getattr(lib, name).restype = getattr(lib, name).restype if name == "ltd_status_string" else C.c_int
    _lib = lib
    return lib


class LtdError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = load().ltd_status_string(code).decode()
        super().__init__(f"{where}: {msg} (status {code})")
        self.code = code


def check(code: int, where: str):
    if code != LTD_OK:
        raise LtdError(code, where)
