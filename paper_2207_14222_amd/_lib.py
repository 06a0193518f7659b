"""ctypes binding of ``libusp.so`` (argument marshalling only).

The functions here have the same names and arguments as the C ABI declared in
``include/usp.h``.  Loading fails loudly when the library has not been built:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libusp.so")

USP_OK, USP_MAXIT, USP_STAGNATED, USP_DIVERGED = 0, 1, 2, 3
USP_ERR_INVALID, USP_ERR_UNSUPPORTED_SHAPE, USP_ERR_NOT_CONTRACTIVE = -1, -2, -3
USP_ERR_HIP, USP_ERR_NAN, USP_ERR_WORKSPACE = -4, -5, -6
USP_C64, USP_C128 = 0, 1
USP_FLAG_REFINE = 1
USP_FLAG_ANTISYM = 2
USP_BIAS_COMPLEX, USP_BIAS_REAL = 0, 1
USP_KRYLOV_BICGSTAB, USP_KRYLOV_GMRES, USP_KRYLOV_CG = 1, 2, 3

STATUS_NAMES = {0: "converged", 1: "maxit", 2: "stagnated", 3: "diverged", -1: "invalid",
                -2: "unsupported_shape", -3: "not_contractive", -4: "hip_error", -5: "nan", -6: "workspace"}

EXPORTS = ["usp_workspace_bytes", "usp_prepare_operator", "usp_solve", "usp_iterate", "usp_residual",
           "usp_destroy", "usp_last_error", "usp_smallest_circle", "usp_canonical_fields",
           "usp_canonical_helmholtz", "usp_canonical_diffusion", "usp_profile", "usp_get_plan", "usp_set_plan",
           "usp_autotune", "usp_canonical_pantograph", "usp_batch_workspace_bytes", "usp_solve_batched",
           "usp_autotune_batched", "usp_nn_conv3d", "usp_nn_wgrad_workspace", "usp_nn_conv3d_wgrad",
           "usp_nn_pool2", "usp_nn_upsample2", "usp_nn_channel_copy", "usp_nn_relu_backward", "usp_nn_add",
           "usp_nn_features", "usp_nn_loss", "usp_nn_adam", "usp_nn_pack_weights", "usp_nn_to_bf16",
           "usp_nn_pred_to_field", "usp_krylov_workspace_bytes", "usp_solve_krylov", "usp_apply_precond",
           "usp_canonical_flux", "usp_flux_workspace_bytes", "usp_flux_solve", "usp_flux_residual",
           "usp_flux_refined_workspace_bytes", "usp_flux_solve_refined",
           "usp_eigs_workspace_bytes", "usp_eigs", "usp_hermitian_eig", "usp_stream_copy",
           "usp_canonical_schrodinger", "usp_residual_static"]
USP_NPASS = 11
PASS_NAMES = ["x_fused", "m_fwd", "sym", "m_inv", "x_first", "r_fwd", "r_mfwd", "r_sym", "r_minv", "r_inv", "reduce"]


class usp_symbol(ct.Structure):
    _fields_ = [("ndim", ct.c_int), ("shape", ct.c_int * 3), ("spacing", ct.c_double * 3),
                ("s", ct.c_double * 2), ("a0", ct.c_double * 2), ("a1", ct.c_double * 2),
                ("a2", ct.c_double * 2), ("nyquist_zero", ct.c_int)]


class usp_plan(ct.Structure):
    _fields_ = [("x_prefetch", ct.c_int), ("w_mid", ct.c_int), ("w_sym", ct.c_int), ("x_stream", ct.c_int),
                ("r_load", ct.c_int)]


class usp_batch_item(ct.Structure):
    _fields_ = [("op", ct.c_void_p), ("y_dev", ct.c_void_p), ("x_dev", ct.c_void_p), ("x_is_guess", ct.c_int),
                ("alpha", ct.c_double), ("tol", ct.c_double), ("maxit", ct.c_int)]


class usp_batch_result(ct.Structure):
    _fields_ = [("iterations", ct.c_int), ("status", ct.c_int), ("rho", ct.c_double), ("t_done_ms", ct.c_double)]


class usp_flux_symbol(ct.Structure):
    _fields_ = [("ndim", ct.c_int), ("n", ct.c_int * 3), ("h", ct.c_double), ("s", ct.c_double * 4),
                ("c", ct.c_double), ("mubar", ct.c_double * 2), ("dibar", (ct.c_double * 2) * 9)]


class usp_gather(ct.Structure):
    _fields_ = [("idx_dev", ct.c_void_p), ("g0_dev", ct.c_void_p), ("g1_dev", ct.c_void_p)]


class UspError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libusp.so (raises if it is missing: the HIP library is mandatory)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built; run `python -m paper_2207_14222_amd.build`")
    L = ct.CDLL(LIB_PATH)
    P, D, I, Z = ct.c_void_p, ct.c_double, ct.c_int, ct.c_size_t
    DP, IP = ct.POINTER(ct.c_double), ct.POINTER(ct.c_int)
    L.usp_workspace_bytes.argtypes = [ct.POINTER(usp_symbol), I, I, ct.POINTER(Z)]
    L.usp_prepare_operator.argtypes = [ct.POINTER(usp_symbol), I, I, P, ct.POINTER(usp_gather), P, Z, P,
                                       ct.POINTER(P)]
    L.usp_solve.argtypes = [P, P, P, I, D, D, I, I, IP, DP, I, DP, I, IP]
    L.usp_iterate.argtypes = [P, P, P, I, D, I, DP, I]
    L.usp_residual.argtypes = [P, P, P, DP, DP, DP]
    L.usp_residual_static.argtypes = [ct.POINTER(usp_symbol), I, P, P, P, DP, DP, DP, P]
    L.usp_destroy.argtypes = [P]
    L.usp_last_error.argtypes = []
    L.usp_last_error.restype = ct.c_char_p
    L.usp_smallest_circle.argtypes = [DP, Z, I, DP, DP]
    L.usp_canonical_fields.argtypes = [P, P, Z, DP, DP, D, I, P, P, P]
    SP = ct.POINTER(usp_symbol)
    L.usp_canonical_helmholtz.argtypes = [DP, Z, I, DP, D, SP, SP, DP, DP]
    L.usp_canonical_diffusion.argtypes = [DP, Z, D, D, D, SP, SP, DP, DP]
    L.usp_canonical_schrodinger.argtypes = [DP, Z, D, D, SP, SP, DP, DP]
    L.usp_profile.argtypes = [P, P, P, D, I, DP, DP]
    PP = ct.POINTER(usp_plan)
    L.usp_get_plan.argtypes = [P, PP]
    L.usp_set_plan.argtypes = [P, PP]
    L.usp_autotune.argtypes = [P, P, P, D, I, PP]
    L.usp_stream_copy.argtypes = [P, P, Z, P]
    BI = ct.POINTER(usp_batch_item)
    L.usp_batch_workspace_bytes.argtypes = [BI, I, ct.POINTER(Z)]
    L.usp_solve_batched.argtypes = [BI, I, I, I, P, Z, P, I, ct.POINTER(usp_batch_result), DP]
    L.usp_autotune_batched.argtypes = [BI, I, I, P, Z, P, IP]
    F, LG, FP = ct.c_float, ct.c_long, ct.c_void_p
    L.usp_nn_conv3d.argtypes = [P, P, P, P, I, I, I, I, I, I, I, I, I, I, P]
    L.usp_nn_wgrad_workspace.argtypes = [I, I, I, I, I, I, ct.POINTER(Z)]
    L.usp_nn_conv3d_wgrad.argtypes = [P, P, P, P, P, Z, I, I, I, I, I, I, P]
    L.usp_nn_pool2.argtypes = [P, P, I, I, I, I, I, P]
    L.usp_nn_upsample2.argtypes = [P, P, I, I, I, I, I, I, I, P]
    L.usp_nn_channel_copy.argtypes = [P, I, I, P, I, I, I, LG, P]
    L.usp_nn_relu_backward.argtypes = [P, P, P, LG, I, P]
    L.usp_nn_add.argtypes = [P, P, LG, P]
    L.usp_nn_features.argtypes = [P, P, I, I, I, D, D, D, I, D, D, P]
    L.usp_nn_loss.argtypes = [P, P, F, LG, P, P, DP, P]
    L.usp_nn_adam.argtypes = [P, P, P, P, P, LG, F, F, F, F, I, P]
    L.usp_nn_pack_weights.argtypes = [P, P, I, I, I, I, P]
    L.usp_nn_to_bf16.argtypes = [P, P, LG, P]
    L.usp_nn_pred_to_field.argtypes = [P, F, P, LG, P]
    L.usp_krylov_workspace_bytes.argtypes = [P, I, I, ct.POINTER(ct.c_size_t)]
    L.usp_apply_precond.argtypes = [P, P, P, I, P, ct.c_size_t]
    L.usp_solve_krylov.argtypes = [P, I, I, P, P, I, D, I, I, P, ct.c_size_t, IP, DP, I, DP, I, IP]
    L.usp_eigs_workspace_bytes.argtypes = [P, I, I, ct.POINTER(ct.c_size_t)]
    L.usp_eigs.argtypes = [P, I, I, P, D, I, D, I, P, DP, DP, P, ct.c_size_t, IP, IP]
    L.usp_hermitian_eig.argtypes = [I, DP, DP, DP]
    FS = ct.POINTER(usp_flux_symbol)
    L.usp_canonical_flux.argtypes = [DP, DP, DP, I, IP, D, D, FS, DP, DP, DP]
    L.usp_flux_workspace_bytes.argtypes = [FS, I, ct.POINTER(ct.c_size_t)]
    L.usp_flux_solve.argtypes = [FS, I, P, P, P, P, I, D, D, I, I, P, ct.c_size_t, P, IP, DP, I, DP, I, IP]
    L.usp_flux_residual.argtypes = [FS, I, P, P, P, P, P, ct.c_size_t, P, DP]
    L.usp_flux_refined_workspace_bytes.argtypes = [FS, ct.POINTER(ct.c_size_t)]
    L.usp_flux_solve_refined.argtypes = [FS, P, P, P, P, I, D, D, I, I, P, ct.c_size_t, P, IP, DP, I, DP, I, IP]
    L.usp_canonical_pantograph.argtypes = [DP, DP, I, D, D, D, DP, DP, D, SP, DP, ct.POINTER(ct.c_int32), DP, DP,
                                           DP, DP, DP]
    for name in EXPORTS:
        if name != "usp_last_error":
            getattr(L, name).restype = ct.c_int
    _lib = L
    return L


def last_error() -> str:
    return lib().usp_last_error().decode()


def check(rc: int) -> int:
    """Raise UspError for negative return codes; pass solver outcomes through."""
    if rc < 0:
        raise UspError(rc, last_error())
    return rc
