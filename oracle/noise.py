"""Sky, noise and flux -> magnitude (oracle side).

Sec. 2.1: after the PSF, sky flux can be added, Poisson shot noise is added with
the data in electrons (noise = sqrt(counts)), and pixel counts are turned into
magnitudes.  Table 2 lists sky level (default 0) and exposure time per band as
hyper-parameters; Sec. 2.2 gives zero-points per filter.

Readings: shot noise is Gaussian with variance equal to the counts (continuous,
so FP32 and FP64 agree closely; it equals the Poisson law in the c >> 1
regime); the sky is added before the noise and subtracted after it
(sky-subtracted data); a non-positive count gives magnitude +inf.  A second mode
adds Gaussian noise of fixed width directly in magnitude.

The standard normal for pixel p, band b comes from Philox words 0 and 1 of
counter (p, b, TAG_NOISE, 0) through Box-Muller in FP64.
"""
from __future__ import annotations

import numpy as np

from .rng import TAG_NOISE, box_muller_f64, philox4x32_10


def noise_normals(px: np.ndarray, band: int, seed: int) -> np.ndarray:
    w = philox4x32_10(np.asarray(px, dtype=np.int64), band, TAG_NOISE, 0, seed)
    return box_muller_f64(w[0], w[1])


def magnitudes(G: np.ndarray, obs, px: np.ndarray | None = None) -> np.ndarray:
    """G: [B][npx] post-PSF fluxes (10^(-0.4 m) units) -> magnitudes [B][npx]."""
    G = np.asarray(G, dtype=np.float64)
    B, npx = G.shape
    px = np.arange(npx, dtype=np.int64) if px is None else np.asarray(px, dtype=np.int64)
    m = np.empty_like(G)
    with np.errstate(divide="ignore", invalid="ignore"):
        for b in range(B):
            if obs.noise_model == 0:
                m[b] = np.where(G[b] > 0, -2.5 * np.log10(G[b]), np.inf)
            elif obs.noise_model == 1:
                z = noise_normals(px, b, obs.seed)
                m[b] = np.where(G[b] > 0, -2.5 * np.log10(G[b]) + obs.noise_sigma_mag[b] * z, np.inf)
            elif obs.noise_model == 2:
                z = noise_normals(px, b, obs.seed)
                t = obs.exptime[b]
                c = G[b] * t * 10.0 ** (0.4 * obs.zp[b]) + obs.sky[b]
                c2 = c + np.sqrt(np.maximum(c, 0.0)) * z - obs.sky[b]
                m[b] = np.where(c2 > 0, -2.5 * np.log10(c2 / t) + obs.zp[b], np.inf)
            else:
                raise ValueError(obs.noise_model)
    return m
