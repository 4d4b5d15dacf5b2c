"""Hess diagram of pixel colour and magnitude (oracle side).

Sec. 2.1 and 2.5: the pCMD is a 2-D histogram of pixel colour and magnitude
with bins 0.05 mag wide in each dimension (Table 2).  The likelihood's extra
term needs the mean colour and magnitude of the pixels (Sec. 2.5).

Rule (FP64): x = m_blue - m_red, y = m_mag; ix = clamp(floor((x - x0)/dx), 0,
nx - 1) with NaN mapped to bin 0, likewise iy; H[iy][ix] += 1.  Out-of-range
pixels land in the edge bins, so the Hess total equals the pixel count.  The
moments are sums of x and y over pixels whose three magnitudes are finite.
"""
from __future__ import annotations

import numpy as np


def bin_index(t: np.ndarray, n: int) -> np.ndarray:
    """clamp(floor(t), 0, n-1), NaN -> 0."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros(t.shape, dtype=np.int64)
    ok = t >= 0.0
    with np.errstate(invalid="ignore"):
        fl = np.floor(np.where(ok & np.isfinite(t), t, 0.0))
    out = np.where(ok, np.minimum(fl, n - 1), 0).astype(np.int64)
    out = np.where(ok & ~np.isfinite(t), n - 1, out)
    return out


def pixel_bins(mags: np.ndarray, grid: dict, b_blue: int, b_red: int, b_mag: int):
    m = np.asarray(mags, dtype=np.float32).astype(np.float64)
    with np.errstate(invalid="ignore"):
        x = m[b_blue] - m[b_red]
        y = m[b_mag]
        tx = (x - grid["x0"]) / grid["dx"]
        ty = (y - grid["y0"]) / grid["dy"]
    return bin_index(tx, grid["nx"]), bin_index(ty, grid["ny"]), x, y


def hess(mags: np.ndarray, grid: dict, b_blue: int = 0, b_red: int = 1, b_mag: int = 1):
    """mags: [B][npx] (the FP32 values the pipeline stores) -> (H[ny][nx] int64,
    moments [sum x, sum y, n_finite])."""
    ix, iy, x, y = pixel_bins(mags, grid, b_blue, b_red, b_mag)
    H = np.zeros((grid["ny"], grid["nx"]), dtype=np.int64)
    np.add.at(H, (iy, ix), 1)
    m = np.asarray(mags, dtype=np.float32).astype(np.float64)
    fin = np.isfinite(m[b_blue]) & np.isfinite(m[b_red]) & np.isfinite(m[b_mag])
    mom = np.array([x[fin].sum(), y[fin].sum(), float(fin.sum())])
    return H, mom
