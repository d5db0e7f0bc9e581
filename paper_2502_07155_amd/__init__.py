"""MI355X (gfx950) library for the NFFT-like procedure for bandlimited functions
(Kircheis & Potts, Algorithm 4.2) and the classical NFFT (Algorithm 2.1).

The transforms run in hand-written HIP kernels of ``libblnfft.so`` behind a C ABI
(``include/blnfft.h``); this package only marshals torch tensors to that ABI.
"""
from ._lib import BLNFFTError, EXPORTS, LIB_PATH, load  # noqa: F401
from .plan import BatchPlan, Plan, window_transform  # noqa: F401
from .autograd import BandlimitedNFFT, bandlimited_nfft  # noqa: F401

__all__ = ["Plan", "BatchPlan", "window_transform", "BandlimitedNFFT", "bandlimited_nfft", "BLNFFTError",
           "load", "LIB_PATH", "EXPORTS"]
