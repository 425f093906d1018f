"""NFFT hot path on AMD Instinct MI355X: C-ABI library libnfft.so + thin binding.

``Plan(x, N, m, sigma)`` builds a plan on the GPU; ``Plan.forward`` and
``Plan.adjoint`` run the transforms in the library's HIP kernels.
"""
from ._lib import NfftError, load  # noqa: F401
from .nfft import Batch, Plan, calibrate_lds, nfft, nfft_adjoint  # noqa: F401
