"""MI355X (gfx950) sampler of stationary Gaussian random fields by FFT.

Lang & Potthoff, "Fast simulation of Gaussian random fields" (arXiv
1105.2737), Section 3: the two-FFT algorithm and the one-FFT algorithm with
the Hermitian data arrangement, on grids of d = 1, 2, 3 (periodic, or with
Neumann / Dirichlet boundaries), the adjoint of every sampler for training,
batches of fields of uneven sizes, and the covariance estimator of Section 4.
All arithmetic runs in the HIP library libgrf.so (include/grf.h); this
package marshals torch tensors (device memory and streams) into its C ABI.

    plan = Plan((512, 512), cov="matern", sigma=1.0, length_scale=0.1, nu=1.5)
    phi = plan.sample(seed=0, batch=1024)              # [1024, 512, 512] float32 on cuda
    phi = GRFSample.apply(theta, plan, seed, noise)    # differentiable in theta (and noise)
"""
from .api import Plan, Batch, GRFSample, COV_KINDS  # noqa: F401
from ._lib import (GRFError, grf_plan_create, grf_plan_destroy, grf_workspace_size,  # noqa: F401
                   grf_sample, grf_sample_noalloc, grf_sample_stage_count, grf_sample_stage, grf_sample_stage_info,
                   grf_sample_from_noise, grf_noise, grf_backward, grf_debug_philox, grf_debug_spectrum,
                   grf_covariance,
                   grf_last_error, grf_version, GRF_PASS_COL_GEN_INV,
                   GRF_PASS_COL_LOAD_INV, GRF_PASS_COL_FILTER, GRF_PASS_ROW_C2R, GRF_PASS_ROW_R2C_GEN, GRF_PASS_ROW_GEN_C2R,
                   GRF_PASS_R2R_COL_GEN, GRF_PASS_R2R_COL_LOAD, GRF_PASS_R2R_ROW_LOAD, GRF_PASS_R2R_ROW_GEN,
                   GRF_PASS_COL_SEQ_INV, GRF_PASS_SPEC_FILTER,
                   GRF_BC_PERIODIC, GRF_BC_NEUMANN, GRF_BC_DIRICHLET, GRF_DRAW_COUNTER, GRF_DRAW_RECURSIVE)
