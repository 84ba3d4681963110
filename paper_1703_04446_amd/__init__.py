"""MI355X-native Lagrangian Gauss-Newton-Krylov registration hot path.

The computation lives in ``liblaglddmm.so`` (hand-written HIP for gfx950,
built by ``paper_1703_04446_amd.build``); this package is a thin ctypes
binding with the C-ABI's function names.  Importing the package does not
touch the GPU; the library is loaded on first use and a missing library is
an error.
"""

from ._lib import (  # noqa: F401
    LAG_OK, LAG_EINVAL, LAG_EUNSUPPORTED, LAG_EHIP, LAG_ENOMEM, LAG_EBREAKDOWN, LAG_ELINESEARCH, LAG_ETOOLARGE,
    LAG_TRANSPORT, LAG_CONTINUITY, LAG_DIFFUSION, LAG_CURVATURE,
    LagProblem, LagError, Plan, make_problem, load, header_symbols, strerror,
    lag_problem_check, lag_problem_sizes, lag_plan_create, lag_plan_destroy, lag_plan_flags, lag_adjoint_stats,
    lag_trace, lag_transport, lag_pushforward, lag_pushforward_noalloc, lag_jvp, lag_vjp, gn_hessmat,
    spectral_precond_apply, lag_reg_apply, lag_objective, lag_gradient, lag_gradient_at_zero, lag_dot,
    lag_pcg, lag_gn_default_options, lag_gn_solve, lag_profile_enable, lag_profile_read,
    lag_jacobian_assemble, gn_hessmat_assembled, lag_vjp_assembled, lag_gradient_assembled,
    lag_pcg_assembled, lag_pcg_graph, lag_pcg_assembled_graph, lag_gn_step, lag_jacobian_info, lag_restrict_image, lag_prolong_velocity,
    lag_multilevel_solve, lag_resample_to_velocity_grid,
    lag_autotune_bricks, lag_batch_solve,
    LagCnnConfig, Cnn, lag_cnn_default_config, lag_cnn_create, lag_cnn_destroy, lag_cnn_get_params,
    lag_cnn_set_params, lag_cnn_get_grads, lag_cnn_forward, lag_cnn_backward, lag_cnn_adam_step,
)

from . import warmstart  # noqa: F401,E402

LIB_PATH = __import__("os").path.join(__import__("os").path.dirname(__file__), "liblaglddmm.so")
