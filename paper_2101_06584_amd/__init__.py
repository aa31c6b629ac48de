"""DD/TD/QD (double-, triple-, quad-double) matrix multiplication for AMD
Instinct MI355X (gfx950): error-free-transformation kernels on the FP64 vector
ALUs, a split form on the INT8 matrix cores, a batched persistent form and an
autotuner, behind the C ABI in include/mpgemm.h.  This package is the thin
Python binding (PyTorch supplies device memory and streams)."""
from .api import (BatchPlan, DEFAULT_SLICES, MPGemmError, PREC, alloc_workspace, autotune, axpy,  # noqa: F401
                  crt_moduli, dot, dot_raw, dot_workspace, gemv, gemv_raw,
                  autotune_load, autotune_save, autotune_set, batch_autotune, gemm, gemm_noalloc,
                  gemm_noalloc_raw, gemm_raw, grouped, grouped_raw, load, problem_array,
                  make_opts, matmul, num_configs, probe_peak, split_layout, split_stages, tune_slices, vec,
                  vec_raw, version, workspace_bytes)
