"""Python binding of libmfe (stochastic matrix-free equilibration on MI355X).

Argument marshalling only: every step of the computation runs in the HIP kernels of
libmfe.so.  PyTorch supplies device memory and the current stream.  If the library
is not built, importing works but every call raises LibraryMissing.

Entry points (same names as the C ABI in include/mfe.h):
  default_alpha_beta, equilibrate, Plan (plan_create / plan_equilibrate / plan_lsqr),
  lsqr, residual, draw_signs, last_error, version.
"""
from __future__ import annotations

from ._ffi import (  # noqa: F401
    Csr,
    Dense,
    LibraryMissing,
    MfeError,
    Operator,
    Plan,
    check_targets,
    default_alpha_beta,
    draw_signs,
    equilibrate,
    equilibrate_noalloc,
    last_error,
    last_timing,
    library_path,
    lsqr,
    mlp_forward,
    mlp_loss_grad,
    mlp_sizes,
    mlp_train,
    probe_gather,
    probe_gather_sorted,
    probe_stream,
    residual,
    version,
    warmstart_apply,
)
