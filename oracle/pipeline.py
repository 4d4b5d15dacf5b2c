"""The whole forward model and likelihood in the paper's order (oracle side).

Fig. 1 and Sec. 2.1: weighted points -> per-pixel Poisson counts -> dust,
distance, sum -> PSF -> sky and noise -> magnitudes -> Hess -> likelihood
(Sec. 2.5).
"""
from __future__ import annotations

import numpy as np

from . import entries, hess as hess_mod, loglike as ll_mod, noise, psf, sampler


def simulate(lam, flux32, obs, want_counts=False):
    """Full image: returns dict(F=[B][N*N] pre-PSF FP64, G=post-PSF, mags=[B][N*N] FP32)."""
    N = obs.nim
    B = flux32.shape[0]
    F, s = sampler.simulate_flux(lam, flux32, obs, 0, N * N, want_counts)
    if obs.psf is not None and np.asarray(obs.psf).ndim == 4:  # 4 x 4 sub-pixel PSF grid
        G = psf.convolve_periodic_subpixel(F.reshape(B, N, N), obs.psf[:B]).reshape(B, N * N)
    elif obs.psf is not None:
        G = psf.convolve_periodic(F.reshape(B, N, N), obs.psf[:B]).reshape(B, N * N)
    else:
        G = F.copy()
    mags = noise.magnitudes(G, obs)
    return dict(F=F, G=G, mags=mags.astype(np.float32), mags64=mags, counts=s["counts"], red=s["red"])


def evaluate(model, grid, obs, hgrid, data_hess, data_mom, mode=0, eps=0.01, bands=(0, 1, 1)):
    lam, _, f32 = entries.build_entries(model, grid)
    out = simulate(lam, f32, obs)
    H, mom = hess_mod.hess(out["mags"], hgrid, *bands)
    return ll_mod.loglike(H, data_hess, mom, data_mom, mode, eps), H, mom, out


def loglike_multi_cmd(mags, cmds, mode=0, eps=0.01):
    """Joint log-likelihood of several colour-magnitude diagrams of one image: the sum over the
    diagrams of the binned likelihood of each (extends the two-band pCMD of Sec. 2.1 to three
    bands).  cmds: sequence of (bands, hess_grid, data_hess, data_mom)."""
    total = 0.0
    for bands, hgrid, dh, dm in cmds:
        H, mom = hess_mod.hess(mags, hgrid, *bands)
        total += ll_mod.loglike(H, dh, mom, dm, mode, eps)
    return total
