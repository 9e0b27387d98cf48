"""qcpd: derivative and adjoint of a quadratic cone program's solution map on MI355X.

The computation lives in the HIP library libqcpd.so (C-ABI in include/qcpd.h); this package
is its Python binding plus a torch.autograd.Function whose backward is the adjoint.
"""
from ._capi import (QCPD_OK, QCPD_WARN_NOT_CONVERGED, QCPD_WARN_NONDIFF, QCPD_ERR_INVALID_ARG,
                    QCPD_ERR_DIM, QCPD_ERR_CONE, QCPD_ERR_PATTERN, QCPD_ERR_NAN, QCPD_ERR_HIP,
                    QCPD_ERR_OOM, QCPD_PRECOND_NONE, QCPD_PRECOND_JACOBI, QCPD_PRECOND_CUSTOM,
                    QCPD_PRECOND_EQUIL, QCPD_PRECOND_LEARNED, QCPD_FLAG_FALLBACK,
                    QCPD_ENGINE_AUTO, QCPD_ENGINE_GRAPH, QCPD_ENGINE_PERSISTENT,
                    QCPD_SOLVER_LSQR, QCPD_SOLVER_LSMR, QCPD_CHOICE_AUTO, QCPD_CHOICE_OFF,
                    QCPD_CHOICE_ON, LIB_PATH, EXPORTS)
from .api import (Cones, Opts, Info, Handle, QCPDError, qcpd_create, qcpd_jvp, qcpd_vjp,
                  qcpd_destroy, qcpd_status_str, qcpd_opts_default, qcpd_set_opts,
                  qcpd_set_precond, qcpd_get_diagnostics, qcpd_profile_kernels,
                  qcpd_set_launch, qcpd_get_launch, qcpd_get_layout, qcpd_apply,
                  qcpd_proj_dual, qcpd_resolve, ResolveInfo)
from .autograd import (QCPStructure, qcp_solution_map, BatchStructure,
                       batch_solution_map)
from .learned import (LearnedModel, qcpd_features, qcpd_learned_targets, qcpd_set_learned,
                      qcpd_mlp_init, qcpd_mlp_predict, qcpd_mlp_grad, qcpd_mlp_adam)
from .batch import (BatchHandle, qcpd_batch_create, qcpd_batch_jvp, qcpd_batch_vjp,
                    qcpd_batch_set_opts, qcpd_batch_destroy, qcpd_batch_set_launch,
                    qcpd_batch_get_launch)

__all__ = [
    "BatchHandle", "qcpd_batch_create", "qcpd_batch_jvp", "qcpd_batch_vjp", "qcpd_batch_set_opts",
    "qcpd_batch_destroy", "qcpd_batch_set_launch", "qcpd_batch_get_launch", "qcpd_set_launch",
    "qcpd_get_launch", "qcpd_get_layout", "qcpd_apply", "qcpd_proj_dual", "qcpd_resolve",
    "ResolveInfo",
    "QCPStructure", "qcp_solution_map",
    "LearnedModel", "qcpd_features", "qcpd_learned_targets", "qcpd_set_learned", "qcpd_mlp_init",
    "qcpd_mlp_predict", "qcpd_mlp_grad", "qcpd_mlp_adam",
    "Cones", "Opts", "Info", "Handle", "QCPDError", "qcpd_create", "qcpd_jvp", "qcpd_vjp",
    "qcpd_destroy", "qcpd_status_str", "qcpd_opts_default", "qcpd_set_opts",
    "qcpd_set_precond", "qcpd_get_diagnostics", "qcpd_profile_kernels", "LIB_PATH", "EXPORTS",
]
