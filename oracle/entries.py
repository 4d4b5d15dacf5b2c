"""Weighted isochrone entries: theta -> expected stars per pixel (oracle side).

Sec. 2.1: age x [Fe/H] x mass space is divided into discrete points, each
weighted by the star-formation history, the metallicity distribution and the
IMF, and the weights are normalised to sum to Npix.  Sec. 2.2 gives the model
menu: SFH forms S1-S5 (Table 1), metallicity forms M1-M3 with Gaussian weights
on the [Fe/H] grid and points under 1% dropped, the Salpeter IMF (Table 2).

Readings (the paper does not fix these):
* The SFH and the IMF act independently (Sec. 2.2 says SFH and metal abundance
  are modelled independently; mass weights come from the IMF alone).
* IMF weight of a mass point = the IMF integrated over the point's mass bin; bin
  edges are the geometric midpoints between neighbouring points, and the outer
  edges lie half a log-step beyond the first and last points.
* Tau model: time since the onset of star formation t = T - age with
  T = 10^10.2 yr, the upper edge of the paper's age grid; the stars formed in an
  age bin are the SFR integrated over it.
* Gaussian MDF: weight of a grid point = the normal density at that [Fe/H];
  weights are normalised, those under `prune` (1%) are set to zero, and the rest
  renormalised.  Pruned isochrones keep their entries with zero weight.
* Non-parametric SFH: the age weights are 10^logSFH_a and Npix is their sum.
* Sigma lambda = Npix over all entries (the paper's normalisation).

Pins: Salpeter bin integral in closed form, the MDF weights quoted for
sigma = 0.2, the tau-model bin integral against numerical quadrature, and the
sum of lambda (tests/test_oracle_entries.py).
"""
from __future__ import annotations

import numpy as np

T_ONSET_LOG = 10.2    # log10 yr: upper edge of the age grid (Sec. 2.2 age bins)


def imf_bin_edges(mass: np.ndarray) -> np.ndarray:
    """Mass-bin edges around increasing mass points (geometric midpoints)."""
    lm = np.log(np.asarray(mass, dtype=np.float64))
    mid = 0.5 * (lm[1:] + lm[:-1])
    lo = lm[0] - 0.5 * (lm[1] - lm[0])
    hi = lm[-1] + 0.5 * (lm[-1] - lm[-2])
    return np.exp(np.concatenate([[lo], mid, [hi]]))


def salpeter_bin_weight(m_lo, m_hi, alpha: float = 2.35):
    """Integral of m^-alpha over [m_lo, m_hi] (Salpeter IMF, Sec. 2.2)."""
    m_lo = np.asarray(m_lo, dtype=np.float64)
    m_hi = np.asarray(m_hi, dtype=np.float64)
    return (m_lo ** (1.0 - alpha) - m_hi ** (1.0 - alpha)) / (alpha - 1.0)


# Kroupa (2001): xi(m) proportional to m^-0.3 below 0.08 Msun, m^-1.3 on [0.08, 0.5) and m^-2.3
# above, joined continuously (Sec. 2.2 names it as the alternative to Salpeter).
KROUPA_BREAKS = (0.08, 0.5)
KROUPA_SLOPES = (0.3, 1.3, 2.3)


def kroupa_pdf(m):
    """Unnormalised Kroupa IMF, continuous at the breaks (value 1 * m^-0.3 below the first)."""
    m = np.asarray(m, dtype=np.float64)
    b1, b2 = KROUPA_BREAKS
    a0, a1, a2 = KROUPA_SLOPES
    c1 = b1 ** (a1 - a0)            # continuity at b1
    c2 = c1 * b2 ** (a2 - a1)       # continuity at b2
    return np.where(m < b1, m ** -a0, np.where(m < b2, c1 * m ** -a1, c2 * m ** -a2))


def kroupa_bin_weight(m_lo, m_hi):
    """Integral of kroupa_pdf over [m_lo, m_hi], segment by segment."""
    m_lo = np.atleast_1d(np.asarray(m_lo, dtype=np.float64))
    m_hi = np.atleast_1d(np.asarray(m_hi, dtype=np.float64))
    b1, b2 = KROUPA_BREAKS
    a0, a1, a2 = KROUPA_SLOPES
    c1 = b1 ** (a1 - a0)
    c2 = c1 * b2 ** (a2 - a1)
    out = np.zeros_like(m_lo)
    for lo_b, hi_b, c, a in ((0.0, b1, 1.0, a0), (b1, b2, c1, a1), (b2, np.inf, c2, a2)):
        lo = np.maximum(m_lo, lo_b)
        hi = np.minimum(m_hi, hi_b)
        ok = hi > lo
        out[ok] += c * (hi[ok] ** (1.0 - a) - lo[ok] ** (1.0 - a)) / (1.0 - a)
    return out


def imf_weights(grid, alpha: float = 2.35, imf: str = "salpeter") -> np.ndarray:
    """IMF weight of every entry, per isochrone (its own mass bins)."""
    w = np.empty(grid.n_entries, dtype=np.float64)
    for k in range(grid.n_iso):
        idx = np.nonzero(grid.iso_of_entry == k)[0]
        e = imf_bin_edges(grid.mass[idx])
        w[idx] = kroupa_bin_weight(e[:-1], e[1:]) if imf == "kroupa" else salpeter_bin_weight(e[:-1], e[1:], alpha)
    return w


def sfh_age_weights(model, age_edges: np.ndarray) -> np.ndarray:
    """Relative number of stars formed in each age bin (S1-S5, Sec. 2.2)."""
    n_age = len(age_edges) - 1
    a_lo = 10.0 ** np.asarray(age_edges[:-1], dtype=np.float64)
    a_hi = 10.0 ** np.asarray(age_edges[1:], dtype=np.float64)
    T = 10.0 ** T_ONSET_LOG
    if model.sfh == "ssp":
        w = np.zeros(n_age)
        w[model.ssp_age_index] = 1.0
        return w
    if model.sfh == "const":
        return a_hi - a_lo
    if model.sfh == "tau":
        tau = model.tau_gyr * 1e9
        t1 = T - a_hi          # earlier time (older edge)
        t2 = T - a_lo
        return tau * (np.exp(-t1 / tau) - np.exp(-t2 / tau))
    if model.sfh == "dtau":
        tau = model.tau_gyr * 1e9
        t1 = T - a_hi
        t2 = T - a_lo

        def prim(t):            # antiderivative of t exp(-t/tau)
            return -tau * (t + tau) * np.exp(-t / tau)
        return prim(t2) - prim(t1)
    if model.sfh == "nonparam":
        return 10.0 ** np.asarray(model.log_sfh, dtype=np.float64)
    raise ValueError(model.sfh)


def mdf_weights(model, feh_grid: np.ndarray) -> np.ndarray:
    """Weights of the [Fe/H] grid points (M1-M3, Sec. 2.2)."""
    feh_grid = np.asarray(feh_grid, dtype=np.float64)
    if model.mdf == "single":
        w = np.zeros(len(feh_grid))
        w[model.feh_index] = 1.0
        return w
    if model.mdf == "gauss":
        z = (feh_grid - model.feh_mu) / model.feh_sigma
        w = np.exp(-0.5 * z * z)
        w = w / w.sum()
        w = np.where(w < model.mdf_prune, 0.0, w)
        return w / w.sum()
    raise ValueError(model.mdf)


def npix_of(model) -> float:
    if model.sfh == "nonparam":
        return float(np.sum(10.0 ** np.asarray(model.log_sfh, dtype=np.float64)))
    return float(10.0 ** model.log_npix)


def iso_weights(model, grid) -> np.ndarray:
    """SFH x MDF weight of every isochrone (independent factors)."""
    wa = sfh_age_weights(model, grid.age_edges)
    wz = mdf_weights(model, grid.feh_grid)
    return wa[grid.age_index] * wz[grid.feh_index]


def build_entries(model, grid):
    """lambda_i = Npix * w_i / sum(w) with w_i = SFH x MDF x IMF weight, and the
    per-band star flux f_ib = 10^(-0.4 M_ib) (FP64, plus its FP32 copy)."""
    w = iso_weights(model, grid)[grid.iso_of_entry] * imf_weights(grid, model.imf_alpha, getattr(model, "imf", "salpeter"))
    lam = npix_of(model) * w / w.sum()
    flux64 = 10.0 ** (-0.4 * np.asarray(grid.absmag, dtype=np.float64))
    return lam, flux64, flux64.astype(np.float32)
