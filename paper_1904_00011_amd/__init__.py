"""pCMD forward model on MI355X (gfx950): Python side of the C ABI in include/pcmd.h.

The kernels live in libpcmd.so (built from csrc/ by `python -m paper_1904_00011_amd.build`).
This package only marshals arguments; it raises if the library is not built.
"""
from ._lib import (CONV_AUTO, CONV_DIRECT, CONV_FFT, DUST_LOGNORMAL, DUST_NONE, DUST_SCREEN,  # noqa: F401
                   LL_ACCUMULATE, LL_GAUSS_LITERAL, LL_GAUSS_PAPER, LL_POISSON, NOISE_GAUSS_MAG, NOISE_NONE, NOISE_SHOT,
                   SAMPLER_BLOCK, SAMPLER_HYBRID, SAMPLER_POINT, Context, PcmdError, grid_prepare, iso_weights, load)
from .pipeline import Evaluator  # noqa: F401
