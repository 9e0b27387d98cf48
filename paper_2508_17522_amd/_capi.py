"""ctypes declarations of the C-ABI in include/qcpd.h. Loading fails loudly when the HIP
library has not been built: there is no fallback path."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqcpd.so")

c_int32 = ctypes.c_int32
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p


class qcpd_csr(ctypes.Structure):
    _fields_ = [("nrows", c_int32), ("ncols", c_int32), ("nnz", c_int32),
                ("rowptr", c_void_p), ("colind", c_void_p), ("val", c_void_p)]


class qcpd_cones(ctypes.Structure):
    _fields_ = [("n_zero", c_int32), ("n_nonneg", c_int32), ("n_soc", c_int32),
                ("soc_dims", ctypes.POINTER(c_int32)), ("n_psd", c_int32),
                ("psd_orders", ctypes.POINTER(c_int32)), ("n_exp", c_int32),
                ("n_pow", c_int32), ("pow_alpha", ctypes.POINTER(c_double)),
                ("n_dpow", c_int32), ("dpow_alpha", ctypes.POINTER(c_double))]


class qcpd_opts(ctypes.Structure):
    _fields_ = [("tol", c_double), ("max_iter", c_int32), ("precond", c_int32),
                ("graph_chunk", c_int32), ("check_symmetry", c_int32), ("engine", c_int32),
                ("solver", c_int32), ("staged", c_int32), ("deep", c_int32),
                ("nnz_per_lane_F", c_int32), ("nnz_per_lane_FT", c_int32),
                ("lanes_x", c_int32), ("lanes_y", c_int32),
                ("loop_grid", c_int32), ("persist_grid", c_int32), ("equil_sweeps", c_int32)]


class qcpd_info(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("est_residual", c_double), ("rel_residual", c_double),
                ("flags", ctypes.c_uint32), ("ms_total", ctypes.c_float)]


class qcpd_resolve_info(ctypes.Structure):
    _fields_ = [("newton_iters", c_int32), ("lsqr_iters", c_int32), ("residual", c_double),
                ("converged", c_int32)]


QCPD_CHOICE_AUTO = 0
QCPD_CHOICE_OFF = 1
QCPD_CHOICE_ON = 2

QCPD_OK = 0
QCPD_WARN_NOT_CONVERGED = 1
QCPD_WARN_NONDIFF = 2
QCPD_ERR_INVALID_ARG = -1
QCPD_ERR_DIM = -2
QCPD_ERR_CONE = -3
QCPD_ERR_PATTERN = -4
QCPD_ERR_NAN = -5
QCPD_ERR_HIP = -6
QCPD_ERR_OOM = -7

QCPD_ENGINE_AUTO = 0
QCPD_ENGINE_GRAPH = 1
QCPD_ENGINE_PERSISTENT = 2

QCPD_SOLVER_LSQR = 0
QCPD_SOLVER_LSMR = 1

QCPD_PRECOND_NONE = 0
QCPD_PRECOND_JACOBI = 1
QCPD_PRECOND_CUSTOM = 2
QCPD_PRECOND_EQUIL = 3
QCPD_PRECOND_LEARNED = 4

QCPD_FLAG_NOT_CONVERGED = 1
QCPD_FLAG_NONDIFF = 2
QCPD_FLAG_FALLBACK = 4

# learned preconditioner model
QCPD_NFEAT = 12
QCPD_MLP_HIDDEN = 64
QCPD_MLP_PARAMS = (2 * QCPD_NFEAT + QCPD_MLP_HIDDEN * QCPD_NFEAT + QCPD_MLP_HIDDEN
                   + QCPD_MLP_HIDDEN * QCPD_MLP_HIDDEN + QCPD_MLP_HIDDEN + 2 * QCPD_MLP_HIDDEN + 2)

class qcpd_batch_layout(ctypes.Structure):
    _fields_ = [("nprob", c_int32), ("n", ctypes.POINTER(c_int32)), ("m", ctypes.POINTER(c_int32)),
                ("nnz_P", ctypes.POINTER(c_int32)), ("nnz_A", ctypes.POINTER(c_int32)),
                ("cones", ctypes.POINTER(qcpd_cones))]


EXPORTS = ["qcpd_opts_default", "qcpd_create", "qcpd_jvp", "qcpd_vjp", "qcpd_set_opts",
           "qcpd_set_precond", "qcpd_get_diagnostics", "qcpd_profile_kernels", "qcpd_destroy",
           "qcpd_status_str", "qcpd_batch_create", "qcpd_batch_jvp", "qcpd_batch_vjp",
           "qcpd_batch_set_opts", "qcpd_batch_destroy", "qcpd_features", "qcpd_learned_targets",
           "qcpd_set_learned", "qcpd_mlp_init", "qcpd_mlp_predict", "qcpd_mlp_workspace_floats",
           "qcpd_mlp_grad", "qcpd_mlp_adam", "qcpd_set_launch", "qcpd_get_launch",
           "qcpd_batch_set_launch", "qcpd_batch_get_launch", "qcpd_apply",
           "qcpd_mlp_grad_noalloc", "qcpd_get_layout", "qcpd_proj_dual", "qcpd_resolve"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libqcpd.so and declare the signatures. Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_2508_17522_amd.build)")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.qcpd_opts_default.argtypes = [P(qcpd_opts)]
    lib.qcpd_opts_default.restype = None
    lib.qcpd_create.argtypes = [P(c_void_p), P(qcpd_csr), P(qcpd_csr), c_void_p, c_void_p,
                                P(qcpd_cones), c_void_p, c_void_p, c_void_p, P(qcpd_opts),
                                c_void_p]
    lib.qcpd_create.restype = c_int32
    lib.qcpd_jvp.argtypes = [c_void_p] + [c_void_p] * 7 + [P(qcpd_info)]
    lib.qcpd_jvp.restype = c_int32
    lib.qcpd_vjp.argtypes = [c_void_p] + [c_void_p] * 7 + [P(qcpd_info)]
    lib.qcpd_vjp.restype = c_int32
    lib.qcpd_set_opts.argtypes = [c_void_p, P(qcpd_opts)]
    lib.qcpd_set_opts.restype = c_int32
    lib.qcpd_set_precond.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.qcpd_set_precond.restype = c_int32
    lib.qcpd_get_diagnostics.argtypes = [c_void_p] + [c_void_p] * 5
    lib.qcpd_get_diagnostics.restype = c_int32
    lib.qcpd_profile_kernels.argtypes = [c_void_p, c_int32, P(ctypes.c_float)]
    lib.qcpd_profile_kernels.restype = c_int32
    lib.qcpd_destroy.argtypes = [c_void_p]
    lib.qcpd_destroy.restype = None
    lib.qcpd_batch_create.argtypes = [P(c_void_p), P(qcpd_batch_layout)] + [c_void_p] * 11 + \
        [P(qcpd_opts), c_void_p]
    lib.qcpd_batch_create.restype = c_int32
    lib.qcpd_batch_jvp.argtypes = [c_void_p] + [c_void_p] * 7 + [P(qcpd_info)]
    lib.qcpd_batch_jvp.restype = c_int32
    lib.qcpd_batch_vjp.argtypes = [c_void_p] + [c_void_p] * 7 + [P(qcpd_info)]
    lib.qcpd_batch_vjp.restype = c_int32
    lib.qcpd_batch_set_opts.argtypes = [c_void_p, P(qcpd_opts)]
    lib.qcpd_batch_set_opts.restype = c_int32
    lib.qcpd_batch_destroy.argtypes = [c_void_p]
    lib.qcpd_batch_destroy.restype = None
    lib.qcpd_features.argtypes = [c_void_p, c_void_p]
    lib.qcpd_features.restype = c_int32
    lib.qcpd_learned_targets.argtypes = [c_void_p, c_void_p]
    lib.qcpd_learned_targets.restype = c_int32
    lib.qcpd_set_learned.argtypes = [c_void_p, c_void_p]
    lib.qcpd_set_learned.restype = c_int32
    lib.qcpd_mlp_init.argtypes = [c_void_p, c_int32, ctypes.c_uint64, c_void_p, c_void_p]
    lib.qcpd_mlp_init.restype = c_int32
    lib.qcpd_mlp_predict.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]
    lib.qcpd_mlp_predict.restype = c_int32
    lib.qcpd_mlp_workspace_floats.argtypes = [c_int32]
    lib.qcpd_mlp_workspace_floats.restype = ctypes.c_int64
    lib.qcpd_mlp_grad.argtypes = [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                                  c_void_p]
    lib.qcpd_mlp_grad.restype = c_int32
    lib.qcpd_mlp_grad_noalloc.argtypes = [c_void_p, c_void_p, c_int32, c_void_p, c_void_p,
                                          c_void_p]
    lib.qcpd_mlp_grad_noalloc.restype = c_int32
    lib.qcpd_mlp_adam.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                                  ctypes.c_float, c_void_p]
    lib.qcpd_mlp_adam.restype = c_int32
    lib.qcpd_apply.argtypes = [c_void_p, c_int32, c_void_p, c_void_p]
    lib.qcpd_apply.restype = c_int32
    lib.qcpd_proj_dual.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.qcpd_proj_dual.restype = c_int32
    lib.qcpd_resolve.argtypes = [P(qcpd_csr), P(qcpd_csr), c_void_p, c_void_p, P(qcpd_cones),
                                 c_void_p, c_void_p, c_void_p, P(qcpd_opts), c_double, c_int32,
                                 P(qcpd_resolve_info), c_void_p]
    lib.qcpd_resolve.restype = c_int32
    lib.qcpd_set_launch.argtypes = [c_void_p, c_int32, c_int32]
    lib.qcpd_set_launch.restype = c_int32
    lib.qcpd_get_launch.argtypes = [c_void_p, P(c_int32)]
    lib.qcpd_get_launch.restype = c_int32
    lib.qcpd_get_layout.argtypes = [c_void_p, P(c_int32)]
    lib.qcpd_get_layout.restype = c_int32
    lib.qcpd_batch_set_launch.argtypes = [c_void_p, c_int32]
    lib.qcpd_batch_set_launch.restype = c_int32
    lib.qcpd_batch_get_launch.argtypes = [c_void_p, P(c_int32)]
    lib.qcpd_batch_get_launch.restype = c_int32
    lib.qcpd_status_str.argtypes = [c_int32]
    lib.qcpd_status_str.restype = ctypes.c_char_p
    _lib = lib
    return lib
