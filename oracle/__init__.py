"""FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's oracle leg (its CPU baseline
and its error checks against this oracle) may import this package.  It shares no code
with the GPU library.
"""
from .blnfft_oracle import *  # noqa: F401,F403
from .blnfft_oracle import (  # noqa: F401
    adjoint_at, adjoint_nfft, adjoint_shannon, band, default_beta, dense_forward, dense_Psi,
    dense_B, dense_F, dense_D, deconvolve_pad, direct_sum, dirichlet, example51_f,
    exp_approx_nfft, exp_approx_shannon, exp_samples, fig51_frequencies,
    forward_nfft, forward_shannon, gather_nfft, gather_shannon, grad_x_shannon,
    grad_x_from_theta,
    in_truncated_domain, inverse_fft_step, node_offsets, phi_g, phihat1, psi_g, psihat1,
    rel_err_inf, rel_err_l2, scaled_offset, sinc_pi, spread_shannon,
)
