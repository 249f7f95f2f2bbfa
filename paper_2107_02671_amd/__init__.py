"""MI355X (gfx950) implementation of the NNFFT and the fast sinc transform of
Kircheis, Potts, Tasche (arXiv 2107.02671).

The transforms run in the HIP library libnnfft.so (C ABI in include/nnfft.h);
`binding` is its thin ctypes binding.  Import of this package does not load
the library; the first call does, and fails loudly if it is missing.
"""
from . import binding  # noqa: F401
from .binding import (NNFFT_FP32_COMP, NNFFT_FP64_PLAIN, SINC_QUAD_CLENSHAW_CURTIS,  # noqa: F401
                      SINC_QUAD_GAUSS_LEGENDRE, NnfftError, Plan, SincPlan, nnfft_derive_params,
                      nnfft_destroy, nnfft_exec, nnfft_exec_batch, nnfft_info, nnfft_last_error,
                      nnfft_plan, nnfft_profile_kernels, nnfft_profile_start, nnfft_profile_stop, nnfft_quadrature, nnfft_version,
                      sinc_destroy, sinc_exec, sinc_info, sinc_middle, sinc_middle_dry_run, sinc_plan, sinc_sizes, nnfft_autotune, nnfft_set_tuning,
                      nnfft_get_tuning, nnfft_clear_tuning, Server, NNFFT_REQ_NNFFT, NNFFT_REQ_SINC,
                      NfftPlan, nfft_plan, nfft_exec, nfft_adjoint, nfft_destroy, nfft_plan_dry_run,
                      NNFFT_WINDOW_SINH, NNFFT_WINDOW_BSPLINE, NNFFT_WINDOW_ALGEBRAIC,
                      NNFFT_WINDOW_KAISER_BESSEL)

__all__ = ["binding", "Plan", "SincPlan", "NnfftError", "nnfft_plan", "nnfft_exec", "nnfft_exec_batch",
           "nnfft_info", "nnfft_destroy", "nnfft_profile_start", "nnfft_profile_stop", "nnfft_profile_kernels", "nnfft_derive_params", "nnfft_last_error", "nnfft_quadrature", "nnfft_version",
           "sinc_plan", "sinc_exec", "sinc_info", "sinc_sizes", "sinc_destroy", "sinc_middle", "sinc_middle_dry_run", "NNFFT_FP32_COMP", "NNFFT_FP64_PLAIN",
           "SINC_QUAD_GAUSS_LEGENDRE", "SINC_QUAD_CLENSHAW_CURTIS", "nnfft_autotune", "nnfft_set_tuning",
           "nnfft_get_tuning", "nnfft_clear_tuning", "Server", "NNFFT_REQ_NNFFT", "NNFFT_REQ_SINC",
           "NfftPlan", "nfft_plan", "nfft_exec", "nfft_adjoint", "nfft_destroy", "nfft_plan_dry_run",
           "NNFFT_WINDOW_SINH", "NNFFT_WINDOW_BSPLINE", "NNFFT_WINDOW_ALGEBRAIC",
           "NNFFT_WINDOW_KAISER_BESSEL"]
