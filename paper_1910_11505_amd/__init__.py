"""MI355X stochastic-Galerkin diffusion solver (HIP, gfx950).

Thin Python binding over the C ABI of libsgfs.so (include/sg.h).  Every step
of the solve runs in the library's HIP kernels; this package only marshals
arguments and owns device memory through PyTorch tensors.  Importing the
binding does not load the library; the first call does, and fails loudly when
the library has not been built.
"""
from .binding import (  # noqa: F401
    SGError, Problem, SolveOpts, SolveInfo, load_library, library_path,
    sg_setup, sg_setup_q2, sg_sizes, sg_workspace_bytes, sg_bind, sg_rhs, sg_apply, sg_apply_noalloc,
    sg_set_apply, sg_apply_form,
    sg_precond_apply, sg_gmres_workspace_bytes, sg_gmres_solve, sg_export,
    sg_destroy, sg_last_error, SGInstance, CNN, sg_residual, Batch, sg_autotune_apply,
    sg_mg_workspace_bytes, sg_mg_bind,
    sg_cnn_create, sg_cnn_param_counts, sg_cnn_workspace_bytes, sg_cnn_bind, sg_cnn_set_params,
    sg_cnn_get_params, sg_cnn_make_pair, sg_cnn_run, sg_cnn_get_grads, sg_cnn_apply,
    sg_cnn_destroy, sg_cnn_last_error, sg_attach_cnn, sg_cnn_stage_work_doubles,
    sg_cnn_stage_grad, sg_cnn_backward,
    COV, PC, GROUPING, EXPORT,
)
