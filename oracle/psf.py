"""Periodic PSF convolution (oracle side).

Sec. 2.1: the simulated image in each band is convolved with that band's PSF
model.  Readings: the boundary is periodic (the simulated image is a stationary
random field, so there is no edge to darken) and each band's K x K PSF sums to
one.  G_b[y][x] = sum_{u,v} P_b[u][v] F_b[(y - u + h) mod N][(x - v + h) mod N]
with h = (K - 1) / 2, summed in FP64.

Pins: a delta PSF is the identity, total flux is conserved, the result equals an
FFT-based circular convolution and the variance of i.i.d. input scales by
sum P^2 (tests/test_oracle_pipeline.py).
"""
from __future__ import annotations

import numpy as np


def convolve_periodic(F: np.ndarray, psf: np.ndarray) -> np.ndarray:
    """F: [B][N][N], psf: [B][K][K] -> G: [B][N][N] (FP64)."""
    F = np.asarray(F, dtype=np.float64)
    P = np.asarray(psf, dtype=np.float32).astype(np.float64)
    B, N, _ = F.shape
    K = P.shape[-1]
    h = (K - 1) // 2
    G = np.zeros_like(F)
    for b in range(B):
        for u in range(K):
            for v in range(K):
                G[b] += P[b, u, v] * np.roll(F[b], shift=(u - h, v - h), axis=(0, 1))
    return G


def region_of(N: int, grid: int = 4) -> np.ndarray:
    """[N][N] region index r = grid * floor(grid y / N) + floor(grid x / N) of every pixel."""
    idx = (grid * np.arange(N)) // N
    return idx[:, None] * grid + idx[None, :]


def convolve_periodic_subpixel(F: np.ndarray, psf: np.ndarray) -> np.ndarray:
    """The 4 x 4 sub-pixel model (Sec. 2.2): the image is split into a 4 x 4 grid of regions and
    the pixels of region r take the periodic convolution of the whole image with PSF r.
    F: [B][N][N], psf: [B][16][K][K] -> G: [B][N][N] (FP64)."""
    F = np.asarray(F, dtype=np.float64)
    B, N, _ = F.shape
    reg = region_of(N, 4)
    G = np.zeros_like(F)
    for r in range(16):
        Gr = convolve_periodic(F, np.asarray(psf)[:, r])
        G[:, reg == r] = Gr[:, reg == r]
    return G

